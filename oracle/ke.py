"""Element stiffness of the 8-node trilinear hexahedron (Finite Element Analysis
section: the H8 element whose stiffness matrix is precomputed once).

KE = integral over the unit cube of B^T D B, with D the isotropic linear-elastic
matrix for Young's modulus 1 and Poisson ratio nu; the SIMP modulus E_e
multiplies it per element.  Evaluated with an n x n x n Gauss-Legendre rule
(n = 2 integrates the trilinear element exactly).

Local node order a = 0..7 at unit-cube corners
(0,0,0),(1,0,0),(1,1,0),(0,1,0),(0,0,1),(1,0,1),(1,1,1),(0,1,1);
local dof 3a + c.  Voigt strain order: xx, yy, zz, xy, yz, zx (engineering shear).
"""

from __future__ import annotations

import numpy as np

CORNERS = np.array([
    [0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
    [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1],
], dtype=float)


def elasticity_matrix(nu: float, E: float = 1.0) -> np.ndarray:
    """Isotropic 6x6 D in Voigt form with engineering shear strains."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def shape_gradients(xi: float, eta: float, zeta: float) -> np.ndarray:
    """d N_a / d(x, y, z) for the 8 trilinear shape functions on the unit cube
    (the reference cube is the physical element, so the Jacobian is I)."""
    g = np.zeros((8, 3))
    p = (xi, eta, zeta)
    for a in range(8):
        fac = [p[d] if CORNERS[a, d] == 1 else 1.0 - p[d] for d in range(3)]
        dfac = [1.0 if CORNERS[a, d] == 1 else -1.0 for d in range(3)]
        g[a, 0] = dfac[0] * fac[1] * fac[2]
        g[a, 1] = fac[0] * dfac[1] * fac[2]
        g[a, 2] = fac[0] * fac[1] * dfac[2]
    return g


def strain_matrix(xi: float, eta: float, zeta: float) -> np.ndarray:
    """6 x 24 strain-displacement matrix B at a point of the unit cube."""
    g = shape_gradients(xi, eta, zeta)
    B = np.zeros((6, 24))
    for a in range(8):
        dx, dy, dz = g[a]
        c = 3 * a
        B[0, c + 0] = dx
        B[1, c + 1] = dy
        B[2, c + 2] = dz
        B[3, c + 0] = dy
        B[3, c + 1] = dx
        B[4, c + 1] = dz
        B[4, c + 2] = dy
        B[5, c + 0] = dz
        B[5, c + 2] = dx
    return B


def element_stiffness(nu: float = 0.3, order: int = 2) -> np.ndarray:
    """24 x 24 KE for E = 1 on the unit cube, Gauss rule of ``order`` points per axis."""
    pts, wts = np.polynomial.legendre.leggauss(order)
    pts = 0.5 * (pts + 1.0)  # map [-1, 1] -> [0, 1]
    wts = 0.5 * wts
    D = elasticity_matrix(nu)
    KE = np.zeros((24, 24))
    for a, wa in zip(pts, wts):
        for b, wb in zip(pts, wts):
            for c, wc in zip(pts, wts):
                B = strain_matrix(a, b, c)
                KE += (wa * wb * wc) * (B.T @ D @ B)
    return KE


def rigid_body_modes() -> np.ndarray:
    """24 x 6 nodal vectors of the 3 translations and 3 infinitesimal rotations."""
    R = np.zeros((24, 6))
    for a in range(8):
        x, y, z = CORNERS[a]
        R[3 * a:3 * a + 3, 0] = [1, 0, 0]
        R[3 * a:3 * a + 3, 1] = [0, 1, 0]
        R[3 * a:3 * a + 3, 2] = [0, 0, 1]
        R[3 * a:3 * a + 3, 3] = [-y, x, 0]   # rotation about z
        R[3 * a:3 * a + 3, 4] = [0, -z, y]   # rotation about x
        R[3 * a:3 * a + 3, 5] = [z, 0, -x]   # rotation about y
    return R
