"""Pins of the oracle's global system, solve, compliance and sensitivities
(Finite Element Analysis and Optimality Criteria sections)."""

import numpy as np
import pytest

import synth
from oracle import fem, simp
from oracle.ke import element_stiffness

KE = element_stiffness(0.3)


def grid_coords(nx, ny, nz):
    n = np.arange((nx + 1) * (ny + 1) * (nz + 1))
    return np.stack([n % (nx + 1), (n // (nx + 1)) % (ny + 1), n // ((nx + 1) * (ny + 1))], 1).astype(float)


def test_global_rigid_body_modes_in_null_space():
    nx, ny, nz = 4, 3, 2
    X = grid_coords(nx, ny, nz)
    E = np.random.default_rng(0).uniform(0.1, 1.0, nx * ny * nz)
    K = fem.assemble(E, KE, fem.element_dofs(nx, ny, nz), 3 * len(X))
    modes = []
    for t in np.eye(3):
        modes.append(np.tile(t, len(X)))
    for axis in range(3):
        w = np.zeros(3)
        w[axis] = 1.0
        modes.append(np.cross(w, X).ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-13 * np.abs(m).max()


def test_assembled_equals_elementwise_product():
    p = synth.config_small()
    E = np.random.default_rng(1).uniform(1e-3, 1.0, p.nel)
    edof = fem.element_dofs(p.nelx, p.nely, p.nelz)
    u = synth.random_vector(2, p.ndof)
    K = fem.assemble(E, KE, edof, p.ndof)
    np.testing.assert_allclose(K @ u, fem.apply_K(E, KE, edof, u), atol=1e-12)


def test_patch_test_linear_field_reproduced():
    """Uniform E, a linear displacement prescribed on every boundary node: the
    interior solution is the same linear field and every element strain is uniform."""
    nx, ny, nz = 4, 3, 3
    X = grid_coords(nx, ny, nz)
    rng = np.random.default_rng(3)
    A, b = rng.normal(size=(3, 3)), rng.normal(size=3)
    exact = (X @ A.T + b).ravel()
    onb = ((X[:, 0] == 0) | (X[:, 0] == nx) | (X[:, 1] == 0) | (X[:, 1] == ny)
           | (X[:, 2] == 0) | (X[:, 2] == nz))
    fixed = (3 * np.nonzero(onb)[0][:, None] + np.arange(3)).ravel()
    K = fem.assemble(np.ones(nx * ny * nz), KE, fem.element_dofs(nx, ny, nz), 3 * len(X))
    u = fem.solve(K, np.zeros(3 * len(X)), fixed, exact[fixed])
    np.testing.assert_allclose(u, exact, atol=1e-12)


def test_uniaxial_bar_exact_elongation():
    """Bar along x with roller supports on the three symmetry planes and a uniform
    end traction: delta = F L / (E A) exactly (the linear field is in the element space)."""
    nx, ny, nz = 6, 2, 3
    E0, F = 2.5, 1.7
    X = grid_coords(nx, ny, nz)
    nn = len(X)
    fixed = np.concatenate([3 * np.nonzero(X[:, 0] == 0)[0] + 0,
                            3 * np.nonzero(X[:, 1] == 0)[0] + 1,
                            3 * np.nonzero(X[:, 2] == 0)[0] + 2])
    f = np.zeros(3 * nn)
    # consistent nodal forces of a uniform traction F/(ny nz) on the x = nx face
    t = F / (ny * nz)
    for j in range(ny):
        for k in range(nz):
            for dj in (0, 1):
                for dk in (0, 1):
                    n = nx + (nx + 1) * ((j + dj) + (ny + 1) * (k + dk))
                    f[3 * n] += t / 4.0
    K = fem.assemble(np.full(nx * ny * nz, E0), KE, fem.element_dofs(nx, ny, nz), 3 * nn)
    u = fem.solve(K, f, fixed)
    tip = X[:, 0] == nx
    np.testing.assert_allclose(u[3 * np.nonzero(tip)[0]], F * nx / (E0 * ny * nz), rtol=1e-11)


def tip_ratio(n):
    """Cantilever L/h = 10, square section h = n elements, tip load spread over the
    tip face; returns mean tip deflection / Euler-Bernoulli F L^3 / (3 E I)."""
    nx, ny, nz = 10 * n, n, n
    p = synth.cantilever(nx, ny, nz, volfrac=1.0, rmin=1.5, n_iter=1)
    f = np.zeros(p.ndof)
    J, K_ = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    tipn = p.node_id(nx, J.ravel(), K_.ravel())
    f[3 * tipn + 1] = -1.0 / len(tipn)
    Kg = fem.assemble(np.ones(p.nel), KE, fem.element_dofs(nx, ny, nz), p.ndof)
    u = fem.solve(Kg, f, p.fixed_dofs)
    eb = 1.0 * nx ** 3 / (3.0 * 1.0 * n ** 4 / 12.0)
    return -u[3 * tipn + 1].mean() / eb


def test_cantilever_converges_to_euler_bernoulli():
    r = [tip_ratio(n) for n in (2, 4, 8)]
    err = [abs(1 - v) for v in r]
    assert err[2] < 0.02
    assert err[0] / err[1] > 3.0 and err[1] / err[2] > 3.0


def test_compliance_identities():
    p = synth.config_small()
    o = simp.SimpOracle(p)
    x = synth.random_density(4, p.nel, 0.05, 1.0)
    r = o.step(x)
    K = fem.assemble(r["E"], KE, o.edof, p.ndof)
    c = r["c"]
    assert abs(c - r["u"] @ (K @ r["u"])) < 1e-10 * c
    assert abs(c - np.sum(r["E"] * r["ce"])) < 1e-10 * c
    # equilibrium of the reduced system
    free = fem.free_dofs(p.ndof, p.fixed_dofs)
    res = (K @ r["u"] - p.f)[free]
    assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(p.f)
    assert np.all(r["u"][p.fixed_dofs] == 0.0)


@pytest.mark.parametrize("mode", ["density", "sensitivity"])
def test_sensitivity_matches_finite_differences(mode):
    """Central differences of c, h = 1e-6, on a 4x3x2 grid with a passive element."""
    p = synth.cantilever(4, 3, 2, volfrac=0.4, rmin=1.5, n_iter=1)
    p.mask[5] = 1
    p.filter_mode = mode
    o = simp.SimpOracle(p)
    x = synth.random_density(5, p.nel, 0.2, 0.9)
    x[5] = 0.0
    r = o.step(x)

    def comp(xv):
        E = fem.simp_modulus(o.physical(xv), p.E0, p.Emin, p.penal)
        return fem.compliance(p.f, o.solve(E))

    h = 1e-6
    if mode == "density":
        grad = r["dcf"]
        for j in range(p.nel):
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            fd = (comp(xp) - comp(xm)) / (2 * h)
            assert abs(fd - grad[j]) <= 1e-6 * np.abs(grad).max(), j
    else:
        # raw (unfiltered) sensitivity with respect to the physical density
        for j in range(p.nel):
            if p.mask[j]:
                continue
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            fd = (comp(xp) - comp(xm)) / (2 * h)
            assert abs(fd - r["dc"][j]) <= 1e-6 * np.abs(r["dc"]).max(), j


def test_sampled_rows_equal_assembled_product():
    p = synth.config_obstacle(seed=7)
    p.nelx, p.nely, p.nelz = 9, 5, 4
    p.mask = None
    E = np.random.default_rng(2).uniform(0.01, 1, 180)
    edof = fem.element_dofs(9, 5, 4)
    ndof = 3 * 10 * 6 * 5
    u = synth.random_vector(3, ndof)
    fixed = np.zeros(ndof, bool)
    fixed[np.random.default_rng(4).choice(ndof, 20, replace=False)] = True
    y = fem.apply_K_reduced(E, KE, edof, u, np.nonzero(fixed)[0])
    nodes = np.array([0, 7, 33, 150, 299])
    np.testing.assert_allclose(fem.apply_K_rows(E, KE, (9, 5, 4), u, nodes, fixed),
                               y.reshape(-1, 3)[nodes], atol=1e-13)
