"""Q1 (trilinear, 8-node "B8") hexahedral element stiffness.

Paper Sec. 3: displacement is (tri)linear per element, density is constant per
element; Sec. 7 Test 2 uses B8 bricks.  The element matrix of the unit cube
with E = 1 is K0 (24 x 24); an element of edge h and Young's modulus E has
K_e = E * h * K0 (strain ~ 1/h, volume ~ h^3).

Local node a = i + 2 j + 4 k sits at (i, j, k) in {0,1}^3; local DOF 3 a + c.
Integration: tensor 2x2x2 Gauss rule, exact for these polynomial integrands.
"""
from __future__ import annotations

import numpy as np


def lame(E: float, nu: float):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elasticity_matrix(E: float, nu: float) -> np.ndarray:
    """Isotropic 6x6 matrix, Voigt order xx, yy, zz, yz, xz, xy (engineering shear)."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def local_nodes() -> np.ndarray:
    return np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.int64)


def shape_grad(xi: np.ndarray) -> np.ndarray:
    """Gradients (8, 3) of the trilinear shape functions on the unit cube at xi."""
    g = np.zeros((8, 3))
    for a, (i, j, k) in enumerate(local_nodes()):
        f = [xi[0] if i else 1 - xi[0], xi[1] if j else 1 - xi[1], xi[2] if k else 1 - xi[2]]
        d = [1.0 if i else -1.0, 1.0 if j else -1.0, 1.0 if k else -1.0]
        g[a, 0] = d[0] * f[1] * f[2]
        g[a, 1] = f[0] * d[1] * f[2]
        g[a, 2] = f[0] * f[1] * d[2]
    return g


def shape_values(xi: np.ndarray) -> np.ndarray:
    """Trilinear shape functions (8,) on the unit cube at xi."""
    v = np.empty(8)
    for a, (i, j, k) in enumerate(local_nodes()):
        v[a] = ((xi[0] if i else 1 - xi[0]) * (xi[1] if j else 1 - xi[1])
                * (xi[2] if k else 1 - xi[2]))
    return v


def strain_matrix(grad: np.ndarray) -> np.ndarray:
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = grad[a]
        c = 3 * a
        B[0, c + 0] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1] = gz
        B[3, c + 2] = gy
        B[4, c + 0] = gz
        B[4, c + 2] = gx
        B[5, c + 0] = gy
        B[5, c + 1] = gx
    return B


def gauss_1d(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def k0(nu: float = 0.3, E: float = 1.0, order: int = 2) -> np.ndarray:
    """Unit-cube element stiffness: sum over Gauss points of B^T D B w."""
    D = elasticity_matrix(E, nu)
    x, w = gauss_1d(order)
    K = np.zeros((24, 24))
    for ix in range(order):
        for iy in range(order):
            for iz in range(order):
                xi = np.array([x[ix], x[iy], x[iz]])
                B = strain_matrix(shape_grad(xi))
                K += (B.T @ D @ B) * (w[ix] * w[iy] * w[iz])
    return 0.5 * (K + K.T)


def rigid_body_modes() -> np.ndarray:
    """(24, 6): three translations and three infinitesimal rotations w x X."""
    X = local_nodes().astype(np.float64) - 0.5
    R = np.zeros((24, 6))
    for a in range(8):
        for c in range(3):
            R[3 * a + c, c] = 1.0
        x, y, z = X[a]
        # rotation about x: (0, -z, y); about y: (z, 0, -x); about z: (-y, x, 0)
        R[3 * a:3 * a + 3, 3] = (0.0, -z, y)
        R[3 * a:3 * a + 3, 4] = (z, 0.0, -x)
        R[3 * a:3 * a + 3, 5] = (-y, x, 0.0)
    return R
