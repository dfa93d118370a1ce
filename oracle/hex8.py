"""Unit hex8 element stiffness for isotropic linear elasticity (oracle, FP64).

Test infrastructure only: nothing in the product path imports this package.

Follows Sec. 3.1 (state equation): K_e is the 24x24 stiffness of a trilinear
hexahedron with nu = 0.3 and unit modulus.  Reading taken here (the paper gives
no more detail): the element is the unit cube [0,1]^3 (h = 1), E = 1, local
node a = dx + 2*dy + 4*dz with (dx,dy,dz) in {0,1}^3, local DOF 3*a + c with
c in {x,y,z}.

Two independent computations are provided:
  * ``ke_exact``   - exact rational integration of B^T C B (Fractions), using
                     that every integrand factorises over the three axes;
  * ``ke_gauss``   - 2x2x2 Gauss-Legendre quadrature in floating point (exact
                     for these polynomial integrands).
"""
from fractions import Fraction
import itertools
import numpy as np

NODE_OFFSETS = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]


def lame(nu, E=1):
    """Lame parameters lambda, mu of an isotropic material."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu


def _int_1d(a, b, da, db):
    """Exact integral over [0,1] of phi_a^(da) * phi_b^(db), phi_0 = 1-t, phi_1 = t."""
    # phi_a(t) = (1-t) if a == 0 else t ; phi_a'(t) = -1 or +1
    if da and db:
        return Fraction((2 * a - 1) * (2 * b - 1))
    if da and not db:
        return Fraction(2 * a - 1, 2)          # int phi_a' phi_b = (2a-1) * 1/2
    if db and not da:
        return Fraction(2 * b - 1, 2)
    return Fraction(1, 3) if a == b else Fraction(1, 6)


def grad_product_integral(a, b, i, j):
    """Exact value of int_{[0,1]^3} d_i N_a * d_j N_b over the unit cube."""
    val = Fraction(1)
    for d in range(3):
        val *= _int_1d(NODE_OFFSETS[a][d], NODE_OFFSETS[b][d], d == i, d == j)
    return val


def ke_exact(nu=Fraction(3, 10)):
    """K_e as a 24x24 list of Fractions (unit cube, E = 1).

    K[3a+i, 3b+j] = lam * G(a,b,i,j) + mu * G(a,b,j,i) + mu * delta_ij * sum_k G(a,b,k,k),
    with G(a,b,i,j) = int d_i N_a d_j N_b: the standard isotropic bilinear form
    lam div u div v + 2 mu eps(u):eps(v) written in components.
    """
    nu = Fraction(nu)
    lam, mu = lame(nu, Fraction(1))
    K = [[Fraction(0)] * 24 for _ in range(24)]
    for a in range(8):
        for b in range(8):
            lap = sum(grad_product_integral(a, b, k, k) for k in range(3))
            for i in range(3):
                for j in range(3):
                    v = lam * grad_product_integral(a, b, i, j) \
                        + mu * grad_product_integral(a, b, j, i)
                    if i == j:
                        v += mu * lap
                    K[3 * a + i][3 * b + j] = v
    return K


def ke_gauss(nu=0.3):
    """K_e by 2x2x2 Gauss quadrature with the Voigt B-matrix (float64)."""
    lam, mu = lame(nu, 1.0)
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    g = 0.5 / np.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    K = np.zeros((24, 24))
    for xi in itertools.product(pts, repeat=3):
        dN = np.zeros((8, 3))
        for a, off in enumerate(NODE_OFFSETS):
            phi = [xi[d] if off[d] else 1 - xi[d] for d in range(3)]
            dphi = [1.0 if off[d] else -1.0 for d in range(3)]
            dN[a, 0] = dphi[0] * phi[1] * phi[2]
            dN[a, 1] = phi[0] * dphi[1] * phi[2]
            dN[a, 2] = phi[0] * phi[1] * dphi[2]
        B = np.zeros((6, 24))
        for a in range(8):
            x, y, z = dN[a]
            B[0, 3 * a] = x
            B[1, 3 * a + 1] = y
            B[2, 3 * a + 2] = z
            B[3, 3 * a + 1] = z; B[3, 3 * a + 2] = y     # gamma_yz
            B[4, 3 * a] = z;     B[4, 3 * a + 2] = x     # gamma_xz
            B[5, 3 * a] = y;     B[5, 3 * a + 1] = x     # gamma_xy
        K += 0.125 * B.T @ C @ B                          # weight (1/2)^3
    return K


def ke(nu=0.3):
    """K_e in float64 (from the exact rational form)."""
    return np.array([[float(v) for v in row] for row in ke_exact(Fraction(nu).limit_denominator(10**6))])


def ke_integer(nu=Fraction(3, 10)):
    """(s, K_int) with K_e = K_int / s exactly, K_int integer, s = 720 (1+nu)(1-2nu)."""
    nu = Fraction(nu)
    s = 720 * (1 + nu) * (1 - 2 * nu)
    K = ke_exact(nu)
    Ki = [[v * s for v in row] for row in K]
    assert all(v.denominator == 1 for row in Ki for v in row), "s*K_e is not integral"
    return s, np.array([[int(v) for v in row] for row in Ki], dtype=np.int64)
