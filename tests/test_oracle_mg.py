"""Pins of the multigrid building blocks used as the solver's preconditioner."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fem, mg
from oracle.ke import element_stiffness

KE = element_stiffness(0.3)


def test_prolongation_reproduces_linear_fields():
    df, dc = (6, 5, 3), (3, 3, 2)
    P = mg.prolongation(df, dc)

    def nodal(d, fn, h):
        n = np.arange((d[0] + 1) * (d[1] + 1) * (d[2] + 1))
        X = np.stack([n % (d[0] + 1), (n // (d[0] + 1)) % (d[1] + 1), n // ((d[0] + 1) * (d[1] + 1))], 1) * h
        return np.stack([fn(X), -2 * fn(X), 0.5 * fn(X)], 1).ravel()

    fn = lambda X: 0.3 + 1.1 * X[:, 0] - 0.7 * X[:, 1] + 0.2 * X[:, 2]
    np.testing.assert_allclose(P @ nodal(dc, fn, 2.0), nodal(df, fn, 1.0), atol=1e-14)


def test_rediscretised_equals_galerkin_for_blockwise_constant_moduli():
    dims_f, dims_c = (6, 4, 4), (3, 2, 2)
    rng = np.random.default_rng(0)
    Ec = rng.uniform(0.01, 1.0, np.prod(dims_c))
    # spread each coarse modulus over its 2x2x2 children
    Ef = Ec.reshape(dims_c[2], dims_c[1], dims_c[0]).repeat(2, 0).repeat(2, 1).repeat(2, 2).ravel()
    ndf = 3 * np.prod([d + 1 for d in dims_f])
    ndc = 3 * np.prod([d + 1 for d in dims_c])
    Kf = fem.assemble(Ef, KE, fem.element_dofs(*dims_f), ndf)
    Kc = fem.assemble(mg.coarse_moduli(Ef, dims_f, dims_c), 2.0 * KE, fem.element_dofs(*dims_c), ndc)
    P = mg.prolongation(dims_f, dims_c)
    G = (P.T @ Kf @ P).toarray()
    np.testing.assert_allclose(Kc.toarray(), G, atol=1e-14)
    np.testing.assert_allclose(mg.coarse_moduli(Ef, dims_f, dims_c), Ec, rtol=1e-15)


def test_coarse_moduli_of_odd_grid_count_missing_children_as_zero():
    E = np.ones(3 * 2 * 2)
    Ec = mg.coarse_moduli(E, (3, 2, 2), (2, 1, 1))
    np.testing.assert_allclose(Ec, [1.0, 0.5])


def setup_vcycle(seed=0, degrees=(2, None)):
    p = synth.cantilever(12, 6, 6, volfrac=0.3, rmin=1.5, n_iter=1)
    x = synth.random_density(seed, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    per_level = degrees[2] if len(degrees) > 2 else None
    return p, E, mg.VCycle(p, E, KE, degree=degrees[0], coarse_degree=degrees[1], max_coarse_dof=300,
                           level_degrees=per_level)


# (finest-level degree, coarser-level degree[, per-level degrees]); None: the
# same on every level
DEGREES = [(2, None), (1, 4), (3, 1), (1, 4, [2, 6])]


@pytest.mark.parametrize("degrees", DEGREES)
def test_vcycle_is_symmetric(degrees):
    p, E, V = setup_vcycle(degrees=degrees)
    assert len(V.levels) >= 3
    fixed = V.levels[0].fixed
    a = synth.random_vector(1, p.ndof)
    b = synth.random_vector(2, p.ndof)
    a[fixed] = b[fixed] = 0
    Ma, Mb = V.apply(a), V.apply(b)
    assert abs(Ma @ b - a @ Mb) < 1e-10 * abs(Ma @ b)
    assert a @ Ma > 0


@pytest.mark.parametrize("degrees", DEGREES)
def test_mg_pcg_matches_direct_solve(degrees):
    p, E, V = setup_vcycle(3, degrees)
    A = V.levels[0].A
    b = p.f.copy()
    x, it, rr = mg.pcg(A, b, V.apply, rtol=1e-12)
    K = fem.assemble(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), p.ndof)
    u = fem.solve(K, p.f, p.fixed_dofs)
    assert rr <= 1e-12
    np.testing.assert_allclose(x, u, rtol=0, atol=1e-8 * np.abs(u).max())
    assert it < 60


@pytest.mark.parametrize("n", [1, 2])
def test_coarse_fixed_inherits_clamped_face(n):
    p = synth.cantilever(8 * n, 3, 3, volfrac=0.3, rmin=1.5, n_iter=1)
    fixed = np.zeros(p.ndof, bool)
    fixed[p.fixed_dofs] = True
    fc = mg.coarse_fixed(fixed, (8 * n, 3, 3), (4 * n, 2, 2))
    nodes = np.arange(fc.size // 3)
    on_face = nodes % (4 * n + 1) == 0
    assert np.all(fc.reshape(-1, 3)[on_face]) and not np.any(fc.reshape(-1, 3)[~on_face])


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_chebyshev_smoother_error_is_the_scaled_chebyshev_polynomial(k):
    """With a diagonal operator D^-1 A = diag(mu), k Chebyshev steps from x = 0
    leave the error e_k = T_k((theta - mu)/delta) / T_k(theta/delta) e_0
    (Chebyshev semi-iteration on [lo, hi], theta/delta the interval's centre and
    half-width).  T_k comes from numpy's Chebyshev basis, not from the smoother's
    three-term recurrence."""
    from types import SimpleNamespace

    from numpy.polynomial import chebyshev as C

    _, _, V = setup_vcycle()
    hi = V.lam_max
    lo = hi / mg.CHEB_RATIO
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    rng = np.random.default_rng(k)
    mu = np.concatenate([[lo, hi, theta, 0.5 * lo], rng.uniform(1e-3 * hi, hi, 60)])
    d = rng.uniform(0.5, 4.0, mu.size)
    lv = SimpleNamespace(A=sp.diags(mu * d), diag=d)
    b = rng.standard_normal(mu.size)
    e0 = b / (mu * d)
    Tk = C.Chebyshev.basis(k)
    want = Tk((theta - mu) / delta) / Tk(theta / delta) * e0
    got = e0 - V.smooth(lv, b, np.zeros_like(b), k)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14 * np.abs(e0).max())


def test_per_level_degrees_reach_each_level():
    """VCycle(level_degrees=[a, b]) on three levels is the V-cycle with degree a on
    the finest level and b on the middle one, composed here by hand from smooth(),
    the transfers and the coarsest Cholesky solve; it differs from [a, a]."""
    import scipy.linalg as sla

    p, _, _ = setup_vcycle()
    E = fem.simp_modulus(synth.random_density(9, p.nel, 0.3, 1.0), p.E0, p.Emin, p.penal)
    a, b = 1, 5
    V = mg.VCycle(p, E, KE, degree=3, coarse_degree=3, max_coarse_dof=300, level_degrees=[a, b])
    assert len(V.levels) == 3
    L0, L1, _ = V.levels
    r = synth.random_vector(4, p.ndof)
    r[L0.fixed] = 0.0

    x0 = V.smooth(L0, r, np.zeros_like(r), a)
    r1 = V.P[0].T @ (r - L0.A @ x0)
    x1 = V.smooth(L1, r1, np.zeros_like(r1), b)
    x1 = x1 + V.P[1] @ sla.cho_solve(V.coarse, V.P[1].T @ (r1 - L1.A @ x1))
    x1 = V.smooth(L1, r1, x1, b)
    x0 = V.smooth(L0, r, x0 + V.P[0] @ x1, a)

    got = V.apply(r)
    np.testing.assert_allclose(got, x0, rtol=0, atol=1e-13 * np.abs(x0).max())
    other = mg.VCycle(p, E, KE, degree=3, coarse_degree=3, max_coarse_dof=300, level_degrees=[a, a]).apply(r)
    assert np.abs(other - got).max() > 1e-3 * np.abs(got).max()


def _jacobi_scaled_lambda_max(p, xphys):
    """lambda_max(D^-1 A) of the finest-level operator (identity rows on fixed
    dofs), by scipy's Lanczos on D^-1/2 A D^-1/2, relative to the element bound."""
    import scipy.sparse.linalg as sla

    E = fem.simp_modulus(xphys, p.E0, p.Emin, p.penal)
    V = mg.VCycle(p, E, KE, degree=1, max_coarse_dof=300)
    A = V.levels[0].A
    s = sp.diags(1.0 / np.sqrt(A.diagonal()))
    lam = sla.eigsh(s @ A @ s, k=1, which="LA", return_eigenvectors=False, tol=1e-8)[0]
    return lam / V.lam_max


def test_smoothing_interval_fractions_of_the_element_bound():
    """The validity range stated for a smoothing interval below the element
    bound: a uniform density sits near 0.58 of it, a filtered SIMP design well
    below 0.8, an isolated solid element in void at the bound itself (its own
    element matrix is the operator there), and no density exceeds it."""
    from oracle import simp

    p = synth.cantilever(16, 8, 8, volfrac=0.3, rmin=1.5, n_iter=1)
    assert abs(_jacobi_scaled_lambda_max(p, np.full(p.nel, 0.3)) - 0.58) < 0.01
    o = simp.SimpOracle(p)
    x, _ = o.trajectory(12)
    assert _jacobi_scaled_lambda_max(p, o.physical(x)) < 0.75
    x = np.full(p.nel, 1e-3)
    x[p.nel // 2 + p.nelx // 2] = 1.0
    ratio = _jacobi_scaled_lambda_max(p, x)
    assert 0.99 < ratio <= 1.0 + 1e-9
    rng = np.random.default_rng(3)
    assert _jacobi_scaled_lambda_max(p, rng.uniform(0.0, 1.0, p.nel)) <= 1.0 + 1e-9
