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
