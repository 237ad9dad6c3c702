"""Flexible preconditioned conjugate gradients with a safeguarded, possibly
non-linear preconditioner and a restart on a fixed SPD fallback (test
infrastructure).

Flexible CG (Notay, SIAM J. Sci. Comput. 22, 2000) replaces the Fletcher-Reeves
ratio of standard PCG by the Polak-Ribiere form
    beta_k = r_{k+1}^T (z_{k+1} - z_k) / (r_k^T z_k),
which keeps CG convergent when the preconditioner changes from one iteration
to the next (a network, or a preconditioner evaluated in lower precision).  A
network output z is accepted only if r^T z > eps ||r|| ||z|| and everything is
finite; otherwise, or after nn_max_iter iterations without convergence, the
solve restarts from the current iterate as standard PCG with the fallback
preconditioner.  Iterations are counted like the GPU path: an iteration is one
update of x and r.
"""

from __future__ import annotations

import numpy as np

SAFE_EPS = 1e-6


def _apply(M, r):
    # a fresh array: a preconditioner may return its argument, which CG updates in place
    return np.array(M(r), dtype=float, copy=True)


def _ok(r, z, rz, beta=0.0):
    if not (np.all(np.isfinite(z)) and np.isfinite(rz) and np.isfinite(beta)):
        return False
    return rz > SAFE_EPS * np.linalg.norm(r) * np.linalg.norm(z)


def fpcg(A, b, M, fallback, x0=None, rtol=1e-10, max_iter=2000, nn_max_iter=200):
    """Returns (x, iterations, relres, fallbacks, learned_iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.astype(float).copy()
    nb = np.linalg.norm(b)
    tol = rtol * nb
    cap = min(max_iter, nn_max_iter)
    r = b - A @ x
    it = 0
    failed = False
    if np.linalg.norm(r) > tol:
        z = _apply(M, r)
        rz = float(r @ z)
        if not _ok(r, z, rz):
            failed = True
        else:
            p = z.copy()
            while True:
                q = A @ p
                alpha = rz / float(p @ q)
                x += alpha * p
                r -= alpha * q
                it += 1
                if np.linalg.norm(r) <= tol or it >= cap:
                    break
                zn = _apply(M, r)
                rzn = float(r @ zn)
                beta = (rzn - float(r @ z)) / rz
                if not _ok(r, zn, rzn, beta):
                    failed = True
                    break
                p = zn + beta * p
                z, rz = zn, rzn
    learned = it
    fallbacks = 0
    if failed or np.linalg.norm(b - A @ x) > tol:
        fallbacks = 1
        r = b - A @ x
        z = _apply(fallback, r)
        p = z.copy()
        rz = float(r @ z)
        while np.linalg.norm(r) > tol and it < max_iter:
            q = A @ p
            alpha = rz / float(p @ q)
            x += alpha * p
            r -= alpha * q
            it += 1
            z = _apply(fallback, r)
            rzn = float(r @ z)
            p = z + (rzn / rz) * p
            rz = rzn
    return x, it, float(np.linalg.norm(b - A @ x) / nb), fallbacks, learned
