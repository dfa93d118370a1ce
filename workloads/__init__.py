"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds no arithmetic of the solver: it only produces densities, Dirichlet
masks, loads and random vectors.  Conventions: node (i,j,k) has index
i + (nx+1)*(j + (ny+1)*k), DOF 3*node + c, element ex + nx*(ey + ny*ez).

Recipes (the paper uses no external dataset, Sec. 6 data statement):
  * uniform cantilever: rho = 0.5 everywhere (Sec. 4.4, E2), x = 0 face
    clamped, unit -z load spread over the nodes (nx, j, 0);
  * Gaussian random field: N(0,1) white noise per element from
    numpy.random.default_rng(seed), separable Gaussian filter with standard
    deviation ``corr_len`` elements (truncate 4 sigma, reflecting boundary),
    standardised, then rho = rho_min + (1 - rho_min) / (1 + exp(-gain * g));
  * random face loads: on one of the five unclamped faces, k random nodes
    with random unit directions, scaled to unit total magnitude;
  * binary-contrast fields (Sec. 4: E1, E5, E10): each element solid
    (rho = 1) with probability V_f, otherwise void at the test floor
    (Bernoulli placement from default_rng(seed); the paper's CuPy draws are
    not reproducible, so its seeds 42 / 7, 11, 13, 17, 19 / 23 name our own
    streams);
  * the deterministic stress fields of E10: a checkerboard of solid and void
    elements, and a layered field (solid lower half in z, void upper half);
  * the mixed near-void field of E10: half the elements near void
    (rho = floor * U(1, 10)), the rest U(0.2, 1), by seed;
  * the two small benchmarks of the auxiliary OC schedule (App. e3_aux),
    which the paper names only: an MBB half-beam (symmetry u_x = 0 on the
    x = 0 face, a roller u_y = u_z = 0 along the bottom edge at x = nx, unit
    -z load along the top edge at x = 0) and a torsion bar (clamped x = 0
    face, unit torque about the bar axis on the x = nx face, nodal forces
    perpendicular to the radius and proportional to it).
"""
import numpy as np


def n_nodes(dims):
    nx, ny, nz = dims
    return (nx + 1) * (ny + 1) * (nz + 1)


def n_elems(dims):
    nx, ny, nz = dims
    return nx * ny * nz


def uniform_rho(dims, value=0.5):
    return np.full(n_elems(dims), float(value))


def cantilever_fixed(dims):
    """uint8 mask over all DOFs, 1 where the node lies on the x = 0 face."""
    nx, ny, nz = dims
    i = np.arange(n_nodes(dims)) % (nx + 1)
    return np.repeat((i == 0).astype(np.uint8), 3)


def edge_load(dims):
    nx, ny, nz = dims
    f = np.zeros(3 * n_nodes(dims))
    for j in range(ny + 1):
        f[3 * (nx + (nx + 1) * j) + 2] = -1.0 / (ny + 1)
    return f


def grf_rho(dims, seed, corr_len=4.0, gain=3.0, rho_min=1e-3):
    from scipy.ndimage import gaussian_filter
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nz, ny, nx))
    g = gaussian_filter(g, sigma=corr_len, mode="reflect", truncate=4.0)
    g = (g - g.mean()) / max(g.std(), 1e-300)
    rho = rho_min + (1.0 - rho_min) / (1.0 + np.exp(-gain * g))
    return rho.reshape(-1)


def random_face_load(dims, rng, max_nodes=8):
    """One load case: k ~ U{1..max_nodes} nodes on a random unclamped face,
    each with a random unit direction; scaled so the nodal force magnitudes
    sum to 1."""
    nx, ny, nz = dims
    face = int(rng.integers(0, 5))
    f = np.zeros(3 * n_nodes(dims))
    k = int(rng.integers(1, max_nodes + 1))
    for _ in range(k):
        a, b = (int(v) for v in rng.integers(0, 10**9, size=2))
        if face == 0:
            i, j, kk = nx, a % (ny + 1), b % (nz + 1)
        elif face == 1:
            i, j, kk = 1 + a % nx, 0, b % (nz + 1)
        elif face == 2:
            i, j, kk = 1 + a % nx, ny, b % (nz + 1)
        elif face == 3:
            i, j, kk = 1 + a % nx, b % (ny + 1), 0
        else:
            i, j, kk = 1 + a % nx, b % (ny + 1), nz
        v = rng.standard_normal(3)
        node = i + (nx + 1) * (j + (ny + 1) * kk)
        f[3 * node:3 * node + 3] += v / np.linalg.norm(v)
    return f / np.linalg.norm(f.reshape(-1, 3), axis=1).sum()


def batch_config(n_systems=32, seed=1000, m_choices=tuple(range(8, 25, 2)), max_loads=4):
    """Uneven cantilever batch: system s has m ~ U(m_choices), mesh (2m, m, m),
    a random-field rho (seed + s, p = 3 in the solver) and 1..max_loads load
    cases.  Returns (dims list, rho list, item_sys list, f list)."""
    rng = np.random.default_rng(seed)
    dims, rhos, item_sys, fs = [], [], [], []
    for s in range(n_systems):
        m = int(rng.choice(m_choices))
        d = (2 * m, m, m)
        dims.append(d)
        rhos.append(grf_rho(d, seed + s))
        for _ in range(int(rng.integers(1, max_loads + 1))):
            item_sys.append(s)
            fs.append(random_face_load(d, rng))
    return dims, rhos, item_sys, fs


def random_vector(n, seed, fixed=None):
    """Standard normal vector, zero on fixed DOFs when a mask is given."""
    v = np.random.default_rng(seed).standard_normal(n)
    if fixed is not None:
        v[np.asarray(fixed).astype(bool)] = 0.0
    return v


def binary_rho(dims, vf, floor, seed):
    """Bernoulli solid/void field: rho = 1 with probability vf, else floor."""
    u = np.random.default_rng(seed).random(n_elems(dims))
    return np.where(u < vf, 1.0, float(floor))


def checkerboard_rho(dims, floor=1e-2):
    nx, ny, nz = dims
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    solid = ((ex + ey + ez) % 2 == 0).transpose(2, 1, 0).reshape(-1)
    return np.where(solid, 1.0, float(floor))


def layered_rho(dims, floor=1e-2):
    """Solid lower half (element layers ez < nz/2), void upper half."""
    nx, ny, nz = dims
    ez = np.arange(n_elems(dims)) // (nx * ny)
    return np.where(ez < nz // 2, 1.0, float(floor))


def mixed_near_void_rho(dims, seed, floor=1e-3):
    rng = np.random.default_rng(seed)
    ne = n_elems(dims)
    void = rng.random(ne) < 0.5
    return np.where(void, floor * rng.uniform(1.0, 10.0, ne), rng.uniform(0.2, 1.0, ne))


def robustness_suite(dims):
    """The ten E10 stress configurations: (label, rho, p)."""
    return [
        ("uniform Vf=0.2", uniform_rho(dims, 0.2), 3.0),
        ("uniform Vf=0.5", uniform_rho(dims, 0.5), 3.0),
        ("uniform Vf=0.8", uniform_rho(dims, 0.8), 3.0),
        ("binary Vf=0.2 p=1.5", binary_rho(dims, 0.2, 1e-2, 7), 1.5),
        ("binary Vf=0.5 p=3", binary_rho(dims, 0.5, 1e-2, 11), 3.0),
        ("binary Vf=0.8 p=4.5", binary_rho(dims, 0.8, 1e-2, 13), 4.5),
        ("checkerboard", checkerboard_rho(dims), 3.0),
        ("layered half solid / half void", layered_rho(dims), 3.0),
        ("binary Vf=0.5 floor 1e-12", binary_rho(dims, 0.5, 1e-12, 17), 3.0),
        ("mixed near-void", mixed_near_void_rho(dims, 19), 3.0),
    ]


def _node_ijk(dims):
    nx, ny, nz = dims
    n = np.arange(n_nodes(dims))
    return n % (nx + 1), (n // (nx + 1)) % (ny + 1), n // ((nx + 1) * (ny + 1))


def mbb_fixed(dims):
    nx, ny, nz = dims
    i, j, k = _node_ijk(dims)
    m = np.zeros((n_nodes(dims), 3), dtype=np.uint8)
    m[i == 0, 0] = 1
    roller = (i == nx) & (k == 0)
    m[roller, 1] = 1
    m[roller, 2] = 1
    return m.reshape(-1)


def mbb_load(dims):
    nx, ny, nz = dims
    i, j, k = _node_ijk(dims)
    f = np.zeros((n_nodes(dims), 3))
    f[(i == 0) & (k == nz), 2] = -1.0 / (ny + 1)
    return f.reshape(-1)


def torsion_load(dims):
    nx, ny, nz = dims
    i, j, k = _node_ijk(dims)
    face = i == nx
    y, z = j[face] - ny / 2.0, k[face] - nz / 2.0
    f = np.zeros((n_nodes(dims), 3))
    f[face, 1] = -z
    f[face, 2] = y
    return f.reshape(-1) / float(np.sum(y * y + z * z))
