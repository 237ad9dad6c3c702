"""Geometric multigrid building blocks, in plain assembled form.

These are not in the paper (which solves K u = f with a direct solver); they
define the preconditioner of the accelerated solver so each of its pieces can be
checked against a plain implementation.

* Hierarchy: each level halves every grid dimension, rounding up; when a fine
  dimension is odd the coarse grid extends half a coarse element past the fine
  domain, the missing fine children counting as zero modulus.
* Coarse element modulus: the mean of the 8 children (missing children = 0).
  Coarse element stiffness: KE scaled by 2^level (3D stiffness of a cube of edge
  h is h times the unit-cube matrix).  With E constant on every 2x2x2 block this
  rediscretised operator equals the Galerkin product P^T K P.
* Transfer: trilinear interpolation P (tensor product of the 1D rule: even fine
  node = coincident coarse node, odd fine node = mean of its two neighbours);
  restriction is P^T.
* Dirichlet data per level: a coarse dof is fixed iff the fine dof at the
  coincident node (clamped into the fine grid) is fixed.  Operators carry
  identity rows/columns at fixed dofs; transfers zero fixed entries on both
  sides.
* Smoother: Chebyshev polynomial in D^-1 A on the interval
  [lam_max / CHEB_RATIO, lam_max] with lam_max the Jacobi-scaled element bound
  lambda_max(diag(KE)^-1 KE) (an upper bound of lambda_max(D^-1 A) for any
  non-negative moduli), or a given fraction of it, same polynomial before and
  after the coarse correction, so the V-cycle is a symmetric operator.
* Coarsest level: direct solve.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem

CHEB_RATIO = 30.0


def hierarchy(nelx, nely, nelz, max_coarse_dof=800, max_levels=12):
    dims = [(nelx, nely, nelz)]
    while len(dims) < max_levels:
        nx, ny, nz = dims[-1]
        if 3 * (nx + 1) * (ny + 1) * (nz + 1) <= max_coarse_dof or min(nx, ny, nz) < 2:
            break
        dims.append(((nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2))
    return dims


def prolong_1d(nf: int, nc: int) -> sp.csr_matrix:
    """(nf+1) x (nc+1) linear interpolation from coarse to fine node positions."""
    rows, cols, vals = [], [], []
    for i in range(nf + 1):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [(i - 1) // 2, (i + 1) // 2]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf + 1, nc + 1))


def prolongation(df, dc) -> sp.csr_matrix:
    """Dof-level P for node numbering x-fastest and dof = 3 n + c."""
    Px, Py, Pz = (prolong_1d(df[a], dc[a]) for a in range(3))
    return sp.kron(Pz, sp.kron(Py, sp.kron(Px, sp.identity(3)))).tocsr()


def coarse_moduli(E: np.ndarray, df, dc) -> np.ndarray:
    nx, ny, nz = df
    Ef = E.reshape(nz, ny, nx)
    pad = np.zeros((2 * dc[2], 2 * dc[1], 2 * dc[0]))
    pad[:nz, :ny, :nx] = Ef
    return pad.reshape(dc[2], 2, dc[1], 2, dc[0], 2).mean(axis=(1, 3, 5)).ravel()


def coarse_fixed(fixed_mask: np.ndarray, df, dc) -> np.ndarray:
    """Per-dof boolean fixed mask on the coarse grid."""
    fm = fixed_mask.reshape(df[2] + 1, df[1] + 1, df[0] + 1, 3)
    I = np.minimum(2 * np.arange(dc[0] + 1), df[0])
    J = np.minimum(2 * np.arange(dc[1] + 1), df[1])
    K = np.minimum(2 * np.arange(dc[2] + 1), df[2])
    return fm[np.ix_(K, J, I)].reshape(-1)


def with_identity_rows(K: sp.csr_matrix, fixed: np.ndarray) -> sp.csr_matrix:
    free = (~fixed).astype(float)
    Mf = sp.diags(free)
    return (Mf @ K @ Mf + sp.diags(fixed.astype(float))).tocsr()


class Level:
    def __init__(self, dims, E, KE, scale, fixed_mask):
        self.dims = dims
        self.E = E
        self.fixed = fixed_mask
        edof = fem.element_dofs(*dims)
        ndof = 3 * (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1)
        self.A = with_identity_rows(fem.assemble(E, KE * scale, edof, ndof), fixed_mask)
        self.diag = self.A.diagonal()


class VCycle:
    """Symmetric V-cycle M ~ A^-1 of the reduced operator with identity rows."""

    def __init__(self, p, E, KE, degree=2, max_coarse_dof=800, levels=None, coarse_degree=None,
                 level_degrees=None, cheb_upper=1.0):
        """degree: Chebyshev steps per pre/post smoothing on the finest level;
        coarse_degree: the same on the coarser levels (None: degree);
        level_degrees: per level, finest first, a degree that replaces those two
        where it is given and positive; cheb_upper: the smoothing interval's top
        as a fraction of the element bound (1: the bound itself)."""
        dims = hierarchy(p.nelx, p.nely, p.nelz, max_coarse_dof)
        if levels is not None:
            dims = dims[:levels]
        fixed = np.zeros(p.ndof, dtype=bool)
        fixed[np.asarray(p.fixed_dofs)] = True
        d = np.diag(KE)
        self.lam_max = cheb_upper * float(np.linalg.eigvalsh(KE / np.sqrt(np.outer(d, d))).max())
        self.degree = degree
        self.coarse_degree = degree if coarse_degree is None else coarse_degree
        self.level_degrees = list(level_degrees or [])
        self.levels, self.P = [], []
        Ecur, fcur = E, fixed
        for l, dl in enumerate(dims):
            self.levels.append(Level(dl, Ecur, KE, 2.0 ** l, fcur))
            if l + 1 < len(dims):
                dc = dims[l + 1]
                fc = coarse_fixed(fcur, dl, dc)
                P = prolongation(dl, dc)
                P = sp.diags((~fcur).astype(float)) @ P @ sp.diags((~fc).astype(float))
                self.P.append(P.tocsr())
                Ecur, fcur = coarse_moduli(Ecur, dl, dc), fc
        self.coarse = sla.cho_factor(self.levels[-1].A.toarray())

    def smooth(self, lv: Level, b, x, degree):
        """Chebyshev smoothing of A x = b from x (degree steps)."""
        hi = self.lam_max
        lo = hi / CHEB_RATIO
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        sigma = theta / delta
        rho = 1.0 / sigma
        r = b - lv.A @ x
        dvec = (r / lv.diag) / theta
        x = x + dvec
        for _ in range(degree - 1):
            r = r - lv.A @ dvec
            rho_new = 1.0 / (2.0 * sigma - rho)
            dvec = rho_new * rho * dvec + (2.0 * rho_new / delta) * (r / lv.diag)
            x = x + dvec
            rho = rho_new
        return x

    def apply(self, r, l=0):
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            return sla.cho_solve(self.coarse, r)
        deg = self.degree if l == 0 else self.coarse_degree
        if l < len(self.level_degrees) and self.level_degrees[l] > 0:
            deg = self.level_degrees[l]
        x = self.smooth(lv, r, np.zeros_like(r), deg)
        res = r - lv.A @ x
        ec = self.apply(self.P[l].T @ res, l + 1)
        x = x + self.P[l] @ ec
        return self.smooth(lv, r, x, deg)


def pcg(A, b, M=None, x0=None, rtol=1e-10, max_iter=2000):
    """Preconditioned CG; stops when ||r|| <= rtol ||b||.  Returns (x, iters, relres)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = r if M is None else M(r)
    pvec = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < max_iter:
        q = A @ pvec
        alpha = rz / (pvec @ q)
        x += alpha * pvec
        r -= alpha * q
        z = r if M is None else M(r)
        rz_new = r @ z
        pvec = z + (rz_new / rz) * pvec
        rz = rz_new
        it += 1
    return x, it, float(np.linalg.norm(r) / nb)
