"""Pins of trilinear prolongation and injection (Sec. 3.3)."""
import numpy as np

from oracle import mesh, transfer


def test_partition_of_unity_even_and_odd():
    for dims in [(4, 4, 2), (5, 3, 7), (15, 7, 3)]:
        Ps = transfer.scalar_prolongation(dims)
        assert np.allclose(Ps @ np.ones(Ps.shape[1]), 1.0, rtol=0, atol=1e-15)


def test_linear_reproduction_even():
    dims = (6, 4, 8)
    cd = transfer.coarse_dims(dims)
    Ps = transfer.scalar_prolongation(dims)

    def coords(d, h):
        nx, ny, nz = d
        k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        return h * i.ravel(), h * j.ravel(), h * k.ravel()
    xf, yf, zf = coords(dims, 1.0)
    xc, yc, zc = coords(cd, 2.0)
    lin = lambda x, y, z: 0.3 + 1.7 * x - 0.4 * y + 2.1 * z
    assert np.abs(Ps @ lin(xc, yc, zc) - lin(xf, yf, zf)).max() < 1e-12


def test_weights_values():
    W = transfer.weights_1d(4)
    assert np.array_equal(W, np.array([[1, 0, 0], [.5, .5, 0], [0, 1, 0], [0, .5, .5], [0, 0, 1]]))
    W = transfer.weights_1d(5)                       # trailing node takes weight 1
    assert np.array_equal(W[5], np.array([0, 0, 1]))


def test_injection_of_clamp():
    dims = (8, 4, 6)
    f = mesh.cantilever_fixed(dims)
    fc = transfer.inject_fixed(f, dims)
    assert np.array_equal(fc, mesh.cantilever_fixed(transfer.coarse_dims(dims)))


def test_vector_prolongation_interleaving():
    dims = (2, 2, 2)
    P = transfer.prolongation(dims)
    Ps = transfer.scalar_prolongation(dims)
    for c in range(3):
        assert abs(P[c::3, c::3] - Ps).max() == 0
        for c2 in range(3):
            if c2 != c:
                assert abs(P[c::3, c2::3]).max() == 0
