"""Global finite-element system of the SIMP problem (Finite Element Analysis and
Optimality Criteria sections).

* element moduli by the modified SIMP law E_e = Emin + rho_e^p (E0 - Emin);
* element -> global dof map (the role of edofMat) and COO triplets (iK, jK,
  sK = E_e KE) converted to CSR;
* fixed displacements applied by eliminating the constrained rows/columns and
  moving their known values to the right-hand side (no penalty);
* a direct sparse solve (SuperLU);
* compliance c = f^T u, element energies ce_e = u_e^T KE u_e and the compliance
  sensitivity dc_e = -p rho_e^(p-1) (E0 - Emin) ce_e.

Numbering: element e = i + nelx (j + nely k), node n = i + (nelx+1)(j + (nely+1)k),
dof 3n + c.  Local node order as in ``oracle.ke``.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ke import CORNERS


def simp_modulus(xphys: np.ndarray, E0: float, Emin: float, penal: float) -> np.ndarray:
    """Modified SIMP interpolation E = Emin + rho^p (E0 - Emin)."""
    return Emin + xphys ** penal * (E0 - Emin)


def element_dofs(nelx: int, nely: int, nelz: int) -> np.ndarray:
    """(nel, 24) array of the global dofs of each element in local order."""
    e = np.arange(nelx * nely * nelz)
    i = e % nelx
    j = (e // nelx) % nely
    k = e // (nelx * nely)
    edof = np.zeros((e.size, 24), dtype=np.int64)
    for a in range(8):
        di, dj, dk = (int(v) for v in CORNERS[a])
        n = (i + di) + (nelx + 1) * ((j + dj) + (nely + 1) * (k + dk))
        for c in range(3):
            edof[:, 3 * a + c] = 3 * n + c
    return edof


def assemble(E: np.ndarray, KE: np.ndarray, edof: np.ndarray, ndof: int) -> sp.csr_matrix:
    """K = sum_e E_e KE scattered by the element dof map (COO -> CSR, duplicates summed)."""
    iK = np.repeat(edof, 24, axis=1).ravel()
    jK = np.tile(edof, (1, 24)).ravel()
    sK = (KE.ravel()[None, :] * E[:, None]).ravel()
    return sp.coo_matrix((sK, (iK, jK)), shape=(ndof, ndof)).tocsr()


def free_dofs(ndof: int, fixed: np.ndarray) -> np.ndarray:
    keep = np.ones(ndof, dtype=bool)
    keep[np.asarray(fixed, dtype=np.int64)] = False
    return np.nonzero(keep)[0]


def solve(K: sp.csr_matrix, f: np.ndarray, fixed: np.ndarray, fixed_values=None) -> np.ndarray:
    """u with u[fixed] = fixed_values (default 0) and K_ff u_f = f_f - K_fc u_c."""
    ndof = K.shape[0]
    fixed = np.asarray(fixed, dtype=np.int64)
    free = free_dofs(ndof, fixed)
    u = np.zeros(ndof)
    if fixed_values is not None:
        u[fixed] = fixed_values
    rhs = f[free] - K[free][:, fixed] @ u[fixed]
    Kff = K[free][:, free].tocsc()
    u[free] = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A").solve(rhs)
    return u


def apply_K(E: np.ndarray, KE: np.ndarray, edof: np.ndarray, u: np.ndarray) -> np.ndarray:
    """sum_e E_e KE u_e scattered to the global vector (no boundary conditions);
    the element-by-element form of the assembled product, for grids too large to
    assemble."""
    ue = u[edof]                      # (nel, 24)
    ye = (ue @ KE.T) * E[:, None]     # (nel, 24)
    return np.bincount(edof.ravel(), weights=ye.ravel(), minlength=u.size)


def apply_K_reduced(E, KE, edof, u, fixed) -> np.ndarray:
    """The operator the reduced system defines on the full vector: free rows get
    (K_ff u_f) with the constrained entries of u taken as zero, constrained rows
    return u itself (identity rows)."""
    fixed = np.asarray(fixed, dtype=np.int64)
    v = u.copy()
    v[fixed] = 0.0
    y = apply_K(E, KE, edof, v)
    y[fixed] = u[fixed]
    return y


def apply_K_rows(E, KE, dims, u, nodes, fixed_mask=None) -> np.ndarray:
    """Rows of the reduced operator for selected nodes: (len(nodes), 3) array of
    sum over the elements around node n of E_e (KE v_e) at n's local position,
    with v = u zeroed on fixed dofs, and u itself on fixed dofs."""
    nelx, nely, nelz = dims
    v = u.copy()
    if fixed_mask is not None:
        v[fixed_mask] = 0.0
    out = np.zeros((len(nodes), 3))
    for r, n in enumerate(np.asarray(nodes)):
        i = n % (nelx + 1)
        j = (n // (nelx + 1)) % (nely + 1)
        k = n // ((nelx + 1) * (nely + 1))
        for ei in (i - 1, i):
            for ej in (j - 1, j):
                for ek in (k - 1, k):
                    if not (0 <= ei < nelx and 0 <= ej < nely and 0 <= ek < nelz):
                        continue
                    e = ei + nelx * (ej + nely * ek)
                    corner = [i - ei, j - ej, k - ek]
                    a = int(np.nonzero((CORNERS == corner).all(axis=1))[0][0])
                    edof = element_dofs_of(e, dims)
                    out[r] += E[e] * (KE[3 * a:3 * a + 3] @ v[edof])
        if fixed_mask is not None:
            for c in range(3):
                if fixed_mask[3 * n + c]:
                    out[r, c] = u[3 * n + c]
    return out


def element_dofs_of(e: int, dims) -> np.ndarray:
    nelx, nely, _ = dims
    i, j, k = e % nelx, (e // nelx) % nely, e // (nelx * nely)
    d = []
    for a in range(8):
        di, dj, dk = (int(t) for t in CORNERS[a])
        n = (i + di) + (nelx + 1) * ((j + dj) + (nely + 1) * (k + dk))
        d += [3 * n, 3 * n + 1, 3 * n + 2]
    return np.array(d)


def compliance(f: np.ndarray, u: np.ndarray) -> float:
    return float(f @ u)


def element_energy(KE: np.ndarray, edof: np.ndarray, u: np.ndarray) -> np.ndarray:
    """ce_e = u_e^T KE u_e."""
    ue = u[edof]
    return np.einsum("ei,ij,ej->e", ue, KE, ue)


def compliance_sensitivity(xphys, ce, E0, Emin, penal) -> np.ndarray:
    """dc_e = -p rho^(p-1) (E0 - Emin) ce_e (compliance is self-adjoint)."""
    return -penal * xphys ** (penal - 1.0) * (E0 - Emin) * ce
