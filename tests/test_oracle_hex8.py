"""Pins of the oracle's element stiffness (Sec. 3.1, unit hex8, nu = 0.3)."""
from fractions import Fraction
import itertools

import numpy as np

from oracle import hex8


def _linear_field(G):
    """Nodal values of u(x) = G x on the unit cube nodes (local order)."""
    u = []
    for off in hex8.NODE_OFFSETS:
        x = [Fraction(v) for v in off]
        for i in range(3):
            u.append(sum(Fraction(G[i][j]) * x[j] for j in range(3)))
    return u


def _quad(K, u, v):
    return sum(u[a] * K[a][b] * v[b] for a in range(24) for b in range(24))


def test_exact_equals_gauss():
    K = np.array([[float(v) for v in r] for r in hex8.ke_exact()])
    assert np.abs(K - hex8.ke_gauss(0.3)).max() < 1e-15


def test_symmetric_exact():
    K = hex8.ke_exact()
    assert all(K[a][b] == K[b][a] for a in range(24) for b in range(24))


def test_uniform_strain_energy_closed_form():
    """u = G x gives u^T K u = lam (tr eps)^2 + 2 mu eps:eps over unit volume."""
    nu = Fraction(3, 10)
    lam, mu = hex8.lame(nu, Fraction(1))
    K = hex8.ke_exact(nu)
    rng = np.random.default_rng(3)
    for _ in range(6):
        G = [[Fraction(int(v)) for v in row] for row in rng.integers(-5, 6, size=(3, 3))]
        u = _linear_field(G)
        eps = [[(G[i][j] + G[j][i]) / 2 for j in range(3)] for i in range(3)]
        tr = eps[0][0] + eps[1][1] + eps[2][2]
        energy = lam * tr * tr + 2 * mu * sum(eps[i][j] ** 2 for i in range(3) for j in range(3))
        assert _quad(K, u, u) == energy


def test_rigid_body_null_space_and_rank():
    K = hex8.ke_exact()
    modes = []
    for c in range(3):
        modes.append([Fraction(1 if i % 3 == c else 0) for i in range(24)])
    for G in ([[0, -1, 0], [1, 0, 0], [0, 0, 0]], [[0, 0, 1], [0, 0, 0], [-1, 0, 0]],
              [[0, 0, 0], [0, 0, -1], [0, 1, 0]]):
        modes.append(_linear_field(G))
    for m in modes:
        assert all(sum(K[a][b] * m[b] for b in range(24)) == 0 for a in range(24))
    assert np.linalg.matrix_rank(hex8.ke()) == 18


def test_integer_structure():
    s, Ki = hex8.ke_integer()
    assert s == Fraction(1872, 5)
    assert np.abs(Ki).max() <= 88
    assert np.allclose(Ki / float(s), hex8.ke(), rtol=0, atol=1e-16)
    # every entry is exactly representable in BF16 (8 significant bits)
    assert all(abs(int(v)) < 256 for v in Ki.ravel())


def test_positive_semidefinite():
    w = np.linalg.eigvalsh(hex8.ke())
    assert w.min() > -1e-14
    assert (w > 1e-10).sum() == 18
