"""Pins of the oracle's flexible CG: exact-inverse and fixed-preconditioner
special cases, and recovery from preconditioners that fail the safeguard."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fpcg, mg


def laplacian_spd(n=60, seed=0):
    """1D Laplacian with a random positive diagonal shift: SPD, condition ~1e3."""
    rng = np.random.default_rng(seed)
    main = 2.0 + rng.uniform(0.0, 0.01, n)
    A = sp.diags([-np.ones(n - 1), main, -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    b = rng.standard_normal(n)
    return A, b


def test_exact_inverse_converges_in_one_iteration():
    A, b = laplacian_spd()
    Ainv = np.linalg.inv(A.toarray())
    x, it, rel, fb, learned = fpcg.fpcg(A, b, lambda r: Ainv @ r, lambda r: r, rtol=1e-12)
    assert it == 1 and fb == 0 and learned == 1 and rel < 1e-12


def test_fixed_preconditioner_reproduces_standard_pcg():
    # with a fixed SPD preconditioner r_{k+1}^T z_k = 0, so Polak-Ribiere = Fletcher-Reeves
    A, b = laplacian_spd(seed=1)
    d = 1.0 / A.diagonal()
    x1, it1, rel1, fb, learned = fpcg.fpcg(A, b, lambda r: d * r, lambda r: r, rtol=1e-10, nn_max_iter=10**6)
    x2, it2, rel2 = mg.pcg(A, b, M=lambda r: d * r, rtol=1e-10)
    assert fb == 0 and abs(it1 - it2) <= 1
    assert np.abs(x1 - x2).max() <= 1e-8 * np.abs(x2).max()


@pytest.mark.parametrize("bad", ["nan", "zero", "negated"])
def test_failing_preconditioner_falls_back_and_converges(bad):
    A, b = laplacian_spd(seed=2)
    M = {"nan": lambda r: np.full_like(r, np.nan), "zero": lambda r: np.zeros_like(r),
         "negated": lambda r: -r}[bad]
    x, it, rel, fb, learned = fpcg.fpcg(A, b, M, lambda r: r, rtol=1e-10, max_iter=5000)
    assert fb == 1 and learned == 0 and rel <= 1e-10
    xs = np.linalg.solve(A.toarray(), b)
    assert np.abs(x - xs).max() <= 1e-7 * np.abs(xs).max()


def test_stagnating_preconditioner_restarts_after_cap():
    # a valid but weak preconditioner (tiny scaling of r): capped, then the fallback finishes
    A, b = laplacian_spd(seed=3)
    x, it, rel, fb, learned = fpcg.fpcg(A, b, lambda r: 1e-3 * r, lambda r: r, rtol=1e-10,
                                        nn_max_iter=5, max_iter=5000)
    assert learned == 5 and fb == 1 and rel <= 1e-10
