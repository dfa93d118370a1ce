"""3D U-Net reference (oracle, FP64): convolutions, pooling, the network and
its gradients, for checking the device training and inference kernels.

Test infrastructure only.

Not a passage of the paper: the learned warm start is an extension.  The
network maps a node-grid input (channels: density averaged to nodes, load
x/y/z, clamp mask) to a displacement shape, with additive skips:
  e1 = relu(c1(x)); e2 = relu(c2(pool(e1))); e3 = relu(c3(pool(e2)));
  b = relu(c4(pool(e3))); d3 = relu(c5(up(b))) + e3; d2 = relu(c6(up(d3))) + e2;
  d1 = relu(c7(up(d2))) + e1; y = c8(d1)
c1..c7 are 3x3x3 convolutions with zero padding (cross-correlation, as in
deep-learning frameworks), c8 a 1x1x1 convolution; pool = 2x2x2 mean,
up = nearest-neighbour x2.  Arrays are (N, C, D, H, W).
"""
import numpy as np

CHANNELS = [(5, 16), (16, 32), (32, 64), (64, 128), (128, 64), (64, 32), (32, 16), (16, 3)]
KSIZE = [3, 3, 3, 3, 3, 3, 3, 1]


def conv3d(x, w, b):
    """y[n,o] = b[o] + sum_{i, taps} w[o,i,t] x[n,i, v + t - r] (zero padding)."""
    k = w.shape[2]
    r = k // 2
    N, Ci, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (r, r), (r, r), (r, r)))
    y = np.zeros((N, w.shape[0], D, H, W))
    for a in range(k):
        for bb in range(k):
            for c in range(k):
                patch = xp[:, :, a:a + D, bb:bb + H, c:c + W]
                y += np.einsum("oi,nidhw->nodhw", w[:, :, a, bb, c], patch)
    return y + b[None, :, None, None, None]


def conv3d_backward(x, w, dy):
    """Gradients (dx, dw, db) of sum(dy * conv3d(x, w, b))."""
    k = w.shape[2]
    r = k // 2
    N, Ci, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (r, r), (r, r), (r, r)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(k):
        for bb in range(k):
            for c in range(k):
                patch = xp[:, :, a:a + D, bb:bb + H, c:c + W]
                dw[:, :, a, bb, c] = np.einsum("nodhw,nidhw->oi", dy, patch)
                dxp[:, :, a:a + D, bb:bb + H, c:c + W] += np.einsum("oi,nodhw->nidhw",
                                                                    w[:, :, a, bb, c], dy)
    dx = dxp[:, :, r:r + D, r:r + H, r:r + W]
    return dx, dw, dy.sum(axis=(0, 2, 3, 4))


def pool(x):
    N, C, D, H, W = x.shape
    return x.reshape(N, C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(3, 5, 7))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3), 2, axis=4) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=2), 2, axis=3), 2, axis=4)


def up_backward(dy):
    N, C, D, H, W = dy.shape
    return dy.reshape(N, C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(3, 5, 7))


def relu(x):
    return np.maximum(x, 0.0)


def init_params(seed=0, channels=CHANNELS, ksize=KSIZE):
    g = np.random.default_rng(seed)
    params = []
    for (ci, co), k in zip(channels, ksize):
        fan_in = ci * k ** 3
        params.append((g.standard_normal((co, ci, k, k, k)) * np.sqrt(2.0 / fan_in), np.zeros(co)))
    return params


def forward(params, x):
    """Returns (y, cache) for the network described in the module docstring."""
    P = params
    c = {}
    c["x0"] = x
    c["r1"] = relu(conv3d(x, *P[0]))
    e1 = c["r1"]
    c["p1"] = pool(e1)
    c["r2"] = relu(conv3d(c["p1"], *P[1]))
    e2 = c["r2"]
    c["p2"] = pool(e2)
    c["r3"] = relu(conv3d(c["p2"], *P[2]))
    e3 = c["r3"]
    c["p3"] = pool(e3)
    c["r4"] = relu(conv3d(c["p3"], *P[3]))
    c["u4"] = up(c["r4"])
    c["r5"] = relu(conv3d(c["u4"], *P[4]))
    d3 = c["r5"] + e3
    c["u3"] = up(d3)
    c["r6"] = relu(conv3d(c["u3"], *P[5]))
    d2 = c["r6"] + e2
    c["u2"] = up(d2)
    c["r7"] = relu(conv3d(c["u2"], *P[6]))
    d1 = c["r7"] + e1
    c["d1"] = d1
    y = conv3d(d1, *P[7])
    return y, c


def loss_mse(y, t, mask):
    """sum(mask * (y - t)^2) / sum(mask); mask (N, 1, D, H, W) broadcast over channels."""
    m = np.broadcast_to(mask, y.shape)
    return float((m * (y - t) ** 2).sum() / m.sum()), 2.0 * m * (y - t) / m.sum()


def backward(params, cache, dy):
    """Gradients [(dw, db)] of the network for output gradient dy."""
    P, c = params, cache
    g = [None] * 8
    dd1, dw, db = conv3d_backward(c["d1"], P[7][0], dy)
    g[7] = (dw, db)
    de1 = dd1.copy()                                    # skip into d1
    dr7 = dd1 * (c["r7"] > 0)
    du2, dw, db = conv3d_backward(c["u2"], P[6][0], dr7)
    g[6] = (dw, db)
    dd2 = up_backward(du2)
    de2 = dd2.copy()
    dr6 = dd2 * (c["r6"] > 0)
    du3, dw, db = conv3d_backward(c["u3"], P[5][0], dr6)
    g[5] = (dw, db)
    dd3 = up_backward(du3)
    de3 = dd3.copy()
    dr5 = dd3 * (c["r5"] > 0)
    du4, dw, db = conv3d_backward(c["u4"], P[4][0], dr5)
    g[4] = (dw, db)
    dr4 = up_backward(du4) * (c["r4"] > 0)
    dp3, dw, db = conv3d_backward(c["p3"], P[3][0], dr4)
    g[3] = (dw, db)
    de3 = de3 + pool_backward(dp3)
    dr3 = de3 * (c["r3"] > 0)
    dp2, dw, db = conv3d_backward(c["p2"], P[2][0], dr3)
    g[2] = (dw, db)
    de2 = de2 + pool_backward(dp2)
    dr2 = de2 * (c["r2"] > 0)
    dp1, dw, db = conv3d_backward(c["p1"], P[1][0], dr2)
    g[1] = (dw, db)
    de1 = de1 + pool_backward(dp1)
    dr1 = de1 * (c["r1"] > 0)
    _, dw, db = conv3d_backward(c["x0"], P[0][0], dr1)
    g[0] = (dw, db)
    return g


def output_to_dofs(y_n, dims, fixed):
    """Sample output (3, D, H, W) -> DOF vector of the (nx, ny, nz) mesh: the
    channels on the first Nz x Ny x Nx voxels (node (i, j, k) at voxel
    (k, j, i), DOF 3 node + c from channel c), zero on the clamped DOFs."""
    nx, ny, nz = dims
    u = y_n[:, :nz + 1, :ny + 1, :nx + 1].transpose(1, 2, 3, 0).reshape(-1).astype(np.float64)
    u[np.asarray(fixed, dtype=bool)] = 0.0
    return u


def dofs_to_output(g, dims, shape):
    """Adjoint of output_to_dofs for one sample (fixed DOFs already zero in g)."""
    nx, ny, nz = dims
    out = np.zeros(shape)
    out[:, :nz + 1, :ny + 1, :nx + 1] = g.reshape(nz + 1, ny + 1, nx + 1, 3).transpose(3, 0, 1, 2)
    return out


def loss_energy(y, Ks, fs, cstars, dims, fixed):
    """Energy-norm score of the predicted displacement shapes and its output
    gradient.  For sample n, u = output_to_dofs(y[n]); the best multiple of u
    in the energy norm of K (the free-DOF stiffness) is alpha u with
    alpha = f.u / u.K u, and its squared error against the solution u* is
    ||u*||_K^2 - (f.u)^2 / u.K u, where ||u*||_K^2 = f.u* = c (the
    compliance).  Score 1 - (f.u)^2 / (u.K u c): 0 for the exact shape,
    1 for u = 0 (score 1 and gradient -f / c when u.K u is not positive).
    Returns (mean score, gradient of the mean with respect to y)."""
    N = y.shape[0]
    dy = np.zeros(y.shape)
    total = 0.0
    for n in range(N):
        u = output_to_dofs(y[n], dims, fixed)
        Ku = Ks[n] @ u
        a, b, c = fs[n] @ u, u @ Ku, cstars[n]
        if b > 0:
            total += 1.0 - a * a / (b * c)
            g = -(2.0 * a / (b * c)) * (fs[n] - (a / b) * Ku)
        else:
            total += 1.0
            g = -np.asarray(fs[n], dtype=np.float64) / c
        g = np.array(g, dtype=np.float64)
        g[np.asarray(fixed, dtype=bool)] = 0.0
        dy[n] = dofs_to_output(g / N, dims, y.shape[1:])
    return total / N, dy
