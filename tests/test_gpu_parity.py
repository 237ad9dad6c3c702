"""GPU parity: every entry point of the C ABI against the CPU FP64 oracle on the
same seeded inputs (small grids spanning several blocks with ragged tails, plus
sampled outputs at the 160x80x80 size)."""

import functools

import numpy as np
import pytest

import synth
from oracle import fem, filt, mg, oc, simp
from oracle.ke import element_stiffness

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu
KE = element_stiffness(0.3)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ragged_problem(seed=0, dims=(13, 7, 5), rmin=2.0, passive=True):
    """Odd-sized grid, a clamped face plus a few extra fixed dofs, random passive elements."""
    q = synth.cantilever(*dims, volfrac=0.3, rmin=rmin, n_iter=5)
    rng = np.random.default_rng(seed)
    extra = rng.choice(q.ndof, 7, replace=False)
    q.fixed_dofs = np.unique(np.concatenate([q.fixed_dofs, extra])).astype(np.int64)
    q.f = synth.random_vector(seed + 1, q.ndof)
    if passive:
        m = np.zeros(q.nel, np.int8)
        m[rng.random(q.nel) < 0.08] = 1
        m[rng.random(q.nel) < 0.03] = 2
        q.mask = m
    return q


def fixed_mask(p):
    fm = np.zeros(p.ndof, bool)
    fm[p.fixed_dofs] = True
    return fm


CASES = ["small", "ragged", "ragged_odd"]
# the two K.u kernels: element columns in the sum/difference basis (the default)
# and node columns applying the element-matrix rows
KERNELS = {"element": 2, "node": 1}


def make_case(name):
    if name == "small":
        return synth.config_small()
    if name == "ragged":
        return ragged_problem(1, (13, 7, 5))
    return ragged_problem(2, (17, 9, 11), rmin=3.0)


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("case", CASES)
def test_apply_K_matches_oracle(case, kernel):
    p = make_case(case)
    x = synth.random_density(3, p.nel, 0.0, 1.0)
    u = synth.random_vector(4, p.ndof)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    ref = fem.apply_K_reduced(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), u, p.fixed_dofs)
    with topo.Context(p, topo.default_opts(ku_kernel=KERNELS[kernel])) as ctx:
        y = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_K(dev(x), dev(u), y)
        got = host(y)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


# multigrid variants: coarse-level cap, Chebyshev degree on the finest and the
# coarser levels, single-workgroup tail below this many nodes
MG_VARIANTS = {
    "mg140": (140, 2, 2, 0), "mg400": (400, 2, 2, 0), "mg400deg3": (400, 3, 3, 0),
    "mg140deg1": (140, 1, 1, 0), "mg140_tail1024": (140, 2, 2, 1024), "mg140_tail4000": (140, 2, 2, 4000),
    "mg1500": (1500, 2, 2, 0), "mg1500d1c4": (1500, 1, 4, 0), "mg140d1c4_tail1024": (140, 1, 4, 1024),
    # per-level degrees, finest first (the levels not listed take the two above)
    "mg140lev": (140, 1, 4, 0, [1, 2, 3, 6]), "mg140lev_tail1024": (140, 1, 4, 1024, [1, 2, 3, 6]),
}


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precond", list(MG_VARIANTS) + ["jacobi"])
def test_preconditioner_matches_oracle(case, precond, kernel):
    """By default every level runs the per-level kernels; _tail1024 and _tail4000
    run the levels below that many nodes as one single-workgroup launch."""
    p = make_case(case)
    x = synth.random_density(5, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    r = synth.random_vector(6, p.ndof)
    r[fixed_mask(p)] = 0.0
    if precond.startswith("mg"):
        coarse, deg, degc, tail = MG_VARIANTS[precond][:4]
        lev = MG_VARIANTS[precond][4] if len(MG_VARIANTS[precond]) > 4 else []
        V = mg.VCycle(p, E, KE, degree=deg, coarse_degree=degc, max_coarse_dof=coarse, level_degrees=lev)
        ref = V.apply(r)
        opts = topo.default_opts(precond=topo.PRECOND_MG, mg_max_coarse_dof=coarse, cheb_degree=deg,
                                 cheb_degree_coarse=degc, coarse_tail_nodes=tail, ku_kernel=KERNELS[kernel],
                                 cheb_degree_level=lev)
    else:
        K = mg.with_identity_rows(fem.assemble(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), p.ndof),
                                  fixed_mask(p))
        ref = r / K.diagonal()
        opts = topo.default_opts(precond=topo.PRECOND_JACOBI, ku_kernel=KERNELS[kernel])
    with topo.Context(p, opts) as ctx:
        if precond.startswith("mg"):
            assert ctx.mg_levels == len(V.levels)
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(x), dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("upper", [1.0, 0.8, 0.7])
@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("tail", [0, 1024])
@pytest.mark.parametrize("lev", [[1, 2, 4, 6], [2, 3, 1, 5]])
def test_per_level_degrees_on_a_five_level_hierarchy(lev, tail, kernel, upper):
    """33x17x17 at a 140-dof cap coarsens to 5 levels, so each of the 4 listed
    degrees smooths a level of its own (the benchmark's 1, 2, 4, 6 among them);
    upper: the top of the smoothing interval as a fraction of the element bound."""
    p = synth.cantilever(33, 17, 17, volfrac=0.3, rmin=1.5, n_iter=1)
    x = synth.random_density(15, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    r = synth.random_vector(16, p.ndof)
    r[fixed_mask(p)] = 0.0
    V = mg.VCycle(p, E, KE, degree=1, coarse_degree=4, max_coarse_dof=140, level_degrees=lev, cheb_upper=upper)
    assert len(V.levels) == len(lev) + 1
    ref = V.apply(r)
    opts = topo.default_opts(mg_max_coarse_dof=140, cheb_degree=1, cheb_degree_coarse=4, cheb_degree_level=lev,
                             coarse_tail_nodes=tail, ku_kernel=KERNELS[kernel], cheb_upper=upper)
    with topo.Context(p, opts) as ctx:
        assert ctx.mg_levels == len(V.levels)
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(x), dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("degrees", [(2, 2), (1, 4)])
@pytest.mark.parametrize("dims", [(32, 16, 16), (40, 20, 20)])
def test_preconditioner_with_large_coarsest_level_matches_oracle(dims, degrees):
    """Coarsest levels of 675 and 1188 dofs: the blocked Gauss-Jordan inverse
    (64-column panels, ragged last panel) against the oracle's exact coarse solve."""
    p = synth.cantilever(*dims, volfrac=0.3, rmin=1.5, n_iter=1)
    x = synth.random_density(5, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    r = synth.random_vector(6, p.ndof)
    r[fixed_mask(p)] = 0.0
    V = mg.VCycle(p, E, KE, degree=degrees[0], coarse_degree=degrees[1], max_coarse_dof=1500)
    ref = V.apply(r)
    with topo.Context(p, topo.default_opts(mg_max_coarse_dof=1500, cheb_degree=degrees[0],
                                           cheb_degree_coarse=degrees[1])) as ctx:
        assert ctx.mg_levels == len(V.levels)
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(x), dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


@functools.lru_cache(maxsize=1)
def large_vcycle_case():
    """102x72x70 nodes (above the size from which the finest level prolongs per
    coarse cell; odd element counts leave ragged cells on every axis)."""
    p = synth.cantilever(101, 71, 69, volfrac=0.3, rmin=1.5, n_iter=1)
    x = synth.random_density(5, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    r = synth.random_vector(6, p.ndof)
    r[fixed_mask(p)] = 0.0
    V = mg.VCycle(p, E, KE, degree=1, coarse_degree=4, max_coarse_dof=1500)
    return p, x, r, V.apply(r), len(V.levels)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_preconditioner_on_a_large_ragged_grid_matches_oracle(precision, tol):
    p, x, r, ref, nlev = large_vcycle_case()
    prec = topo.PREC_FP64 if precision == "fp64" else topo.PREC_FP32
    with topo.Context(p, topo.default_opts(mg_max_coarse_dof=1500, cheb_degree=1, cheb_degree_coarse=4,
                                           precision=prec)) as ctx:
        assert ctx.mg_levels == nlev
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(x), dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("dims,cap,ncoarse", [((12, 4, 4), 200, 189), ((24, 12, 12), 2000, 1911)])
def test_coarse_inverse_panel_edge_sizes(dims, cap, ncoarse):
    """Coarsest levels just above the one-workgroup inverse (189 dofs: panels of
    64, 64 and 61 columns) and near the 2048-dof limit (1911 dofs: 30 panels, the
    last 55 wide) against the oracle's exact coarse solve."""
    p = synth.cantilever(*dims, volfrac=0.3, rmin=1.5, n_iter=1)
    x = synth.random_density(25, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    r = synth.random_vector(26, p.ndof)
    r[fixed_mask(p)] = 0.0
    V = mg.VCycle(p, E, KE, degree=1, coarse_degree=4, max_coarse_dof=cap)
    assert V.levels[-1].A.shape[0] == ncoarse
    ref = V.apply(r)
    with topo.Context(p, topo.default_opts(mg_max_coarse_dof=cap, cheb_degree=1, cheb_degree_coarse=4)) as ctx:
        assert ctx.mg_levels == len(V.levels)
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(x), dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precond", ["mg", "jacobi"])
def test_solve_matches_direct_solve(case, precond, kernel):
    p = make_case(case)
    x = synth.random_density(7, p.nel, 0.05, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    K = fem.assemble(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), p.ndof)
    f = p.f.copy()
    f[p.fixed_dofs] = 0.0
    uref = fem.solve(K, f, p.fixed_dofs)
    opts = topo.default_opts(rtol=1e-11, max_iters=5000, ku_kernel=KERNELS[kernel],
                             precond=topo.PRECOND_MG if precond == "mg" else topo.PRECOND_JACOBI)
    with topo.Context(p, opts) as ctx:
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        st = ctx.solve(dev(x), u)
        got = host(u)
    assert st["converged"] and st["relres"] <= 1e-11
    # true residual of the GPU solution, computed by the oracle
    free = fem.free_dofs(p.ndof, p.fixed_dofs)
    res = (f - K @ got)[free]
    assert np.linalg.norm(res) <= 2e-11 * np.linalg.norm(f)
    assert np.linalg.norm(got - uref) <= 1e-7 * np.linalg.norm(uref)
    assert abs(f @ got - f @ uref) <= 1e-9 * abs(f @ uref)


@pytest.mark.parametrize("case", CASES)
def test_sensitivity_matches_oracle(case):
    p = make_case(case)
    x = synth.random_density(8, p.nel, 0.0, 1.0)
    u = synth.random_vector(9, p.ndof)
    u[p.fixed_dofs] = 0.0
    edof = fem.element_dofs(p.nelx, p.nely, p.nelz)
    ce_ref = fem.element_energy(KE, edof, u)
    dc_ref = fem.compliance_sensitivity(x, ce_ref, p.E0, p.Emin, p.penal)
    f = p.f.copy()
    f[p.fixed_dofs] = 0.0
    with topo.Context(p) as ctx:
        ce = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        dc = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        c = ctx.sensitivity(dev(x), dev(u), ce, dc)
        ce_g, dc_g = host(ce), host(dc)
    np.testing.assert_allclose(ce_g, ce_ref, rtol=1e-12, atol=1e-14 * np.abs(ce_ref).max())
    np.testing.assert_allclose(dc_g, dc_ref, rtol=1e-12, atol=1e-14 * np.abs(dc_ref).max())
    assert abs(c - f @ u) <= 1e-12 * np.abs(f).sum() * np.abs(u).max()


@pytest.mark.parametrize("rmin", [1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 5.0])
@pytest.mark.parametrize("dims", [(11, 7, 6), (20, 10, 4), (37, 19, 13)])
def test_filter_ops_match_oracle(rmin, dims):
    """Every filter operation against the oracle's sparse H.  Reaches 1-3
    (rmin 1.5-4) run the LDS-tiled stencil (37x19x13: several tiles per axis with
    ragged ends), rmin 1 and 5 the offset-list kernel.  The GPU sums a stencil in
    another order than the sparse product: with sign-mixed inputs (ADJ, SENS on a
    random vector) the rounding error is bounded by n eps (H|v|)_e for n stencil
    points, which is the tolerance besides 1e-13 relative."""
    p = ragged_problem(11, dims, rmin=rmin)
    F = filt.Filter(*dims, rmin, p.mask)
    npts = len(filt.filter_offsets(rmin)[0])
    x = synth.random_density(12, p.nel, 0.0, 1.0)
    g = synth.random_vector(13, p.nel)
    refs = {topo.FILTER_FWD: (F.forward(x), 0.0), topo.FILTER_ADJ: (F.adjoint(g), F.adjoint(np.abs(g))),
            topo.FILTER_SENS: (F.sensitivity(x, g), F.sensitivity(x, np.abs(g))),
            topo.FILTER_VOLW: (F.volume_weights(), 0.0)}
    with topo.Context(p) as ctx:
        out = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        for op, (ref, mag) in refs.items():
            inp = dev(x) if op == topo.FILTER_FWD else dev(g)
            ctx.filter(op, inp, out, aux=dev(x) if op == topo.FILTER_SENS else None)
            got = host(out)
            tol = 1e-13 * np.abs(ref) + 1e-15 * np.abs(ref).max() + 2 * npts * 2.2e-16 * mag
            assert np.all(np.abs(got - ref) <= tol), (op, np.max(np.abs(got - ref) - tol))


@pytest.mark.parametrize("rmin", [2.0, 3.0, 4.0])
def test_filter_deep_tiles_match_oracle(rmin):
    """A grid large enough for the 8-element-deep tiles of the stencil kernel,
    ragged in every axis (100 = 3x32 + 4, 70 = 8x8 + 6, 61 = 7x8 + 5)."""
    dims = (100, 70, 61)
    p = ragged_problem(14, dims, rmin=rmin)
    F = filt.Filter(*dims, rmin, p.mask)
    npts = len(filt.filter_offsets(rmin)[0])
    x = synth.random_density(15, p.nel, 0.0, 1.0)
    g = synth.random_vector(16, p.nel)
    refs = {topo.FILTER_FWD: (F.forward(x), 0.0), topo.FILTER_ADJ: (F.adjoint(g), F.adjoint(np.abs(g))),
            topo.FILTER_SENS: (F.sensitivity(x, g), F.sensitivity(x, np.abs(g)))}
    with topo.Context(p, topo.default_opts(precond=topo.PRECOND_JACOBI)) as ctx:
        out = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        for op, (ref, mag) in refs.items():
            inp = dev(x) if op == topo.FILTER_FWD else dev(g)
            ctx.filter(op, inp, out, aux=dev(x) if op == topo.FILTER_SENS else None)
            got = host(out)
            tol = 1e-13 * np.abs(ref) + 1e-15 * np.abs(ref).max() + 2 * npts * 2.2e-16 * mag
            assert np.all(np.abs(got - ref) <= tol), (op, np.max(np.abs(got - ref) - tol))


@pytest.mark.parametrize("tol,lam_tol", [(1e-12, 1e-10), (1e-15, 1e-13)])
@pytest.mark.parametrize("vol_mode", ["design", "all"])
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("move", [0.2, 0.05])
def test_oc_update_matches_exact_multiplier(seed, move, vol_mode, tol, lam_tol):
    """The multiplier and design against the oracle's exact breakpoint root, with
    the volume target over design elements or over all elements (fixed solids
    counted at 1); a tighter oc_tol launches more multisection passes and
    brings the multiplier closer to the root."""
    p = ragged_problem(20 + seed, (23, 11, 9), rmin=2.0)
    p.move = move
    p.vol_mode = vol_mode
    F = filt.Filter(p.nelx, p.nely, p.nelz, p.rmin, p.mask)
    design = p.mask == 0
    rng = np.random.default_rng(seed)
    x = p.initial_design()
    # current volume near the target so that the move limits leave it reachable
    x[design] = rng.uniform(0.0, 2 * p.volfrac, design.sum())
    x[design & (rng.random(p.nel) < 0.05)] = 0.0
    dc = F.adjoint(-rng.exponential(1.0, p.nel) * 10 ** rng.uniform(-3, 2))
    w = F.volume_weights()
    target = simp.SimpOracle(p).target
    if vol_mode == "all":
        assert target == p.volfrac * p.nel - (p.mask == 2).sum()
    xref, lam_ref = oc.oc_exact(x, dc, w, w, target, p.move, p.eta, design)
    assert abs(w @ xref - target) <= 1e-9 * target
    with topo.Context(p, topo.default_opts(oc_tol=tol)) as ctx:
        xn = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        chg, lam = ctx.oc_update(dev(x), dev(dc), dev(w), xn)
        got = host(xn)
    assert abs(lam - lam_ref) <= lam_tol * lam_ref
    np.testing.assert_allclose(got, xref, atol=1e-10)
    assert np.array_equal(got[~design], x[~design])
    assert abs(chg - np.abs(xref - x).max()) <= 1e-10
    assert abs(w @ got - target) <= 1e-9 * target


def test_oc_update_unreachable_target_moves_to_bounds():
    """Volume far above the target with a small move limit: every design element
    takes its lower bound (the multiplier runs to the top of its bracket)."""
    p = ragged_problem(40, (15, 9, 7), rmin=1.5)
    p.move = 0.05
    F = filt.Filter(p.nelx, p.nely, p.nelz, p.rmin, p.mask)
    design = p.mask == 0
    x = p.initial_design()
    x[design] = np.random.default_rng(1).uniform(0.6, 1.0, design.sum())
    dc = F.adjoint(-np.random.default_rng(2).exponential(1.0, p.nel))
    w = F.volume_weights()
    with topo.Context(p) as ctx:
        xn = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        ctx.oc_update(dev(x), dev(dc), dev(w), xn)
        got = host(xn)
    np.testing.assert_allclose(got[design], np.maximum(0.0, x[design] - p.move), atol=1e-12)


def run_gpu_trajectory(p, n_iter, **opt):
    opts = topo.default_opts(rtol=1e-11, max_iters=5000, **opt)
    with topo.Context(p, opts) as ctx:
        x = dev(p.initial_design())
        stats = ctx.iterate(x, n_iter)
        return host(x), stats


@pytest.mark.parametrize("precond", ["mg", "jacobi"])
def test_iterate_matches_oracle_trajectory_small_cantilever(precond):
    p = synth.config_small()
    xo, hist = simp.SimpOracle(p).trajectory()
    xg, stats = run_gpu_trajectory(p, p.n_iter,
                                   precond=topo.PRECOND_MG if precond == "mg" else topo.PRECOND_JACOBI)
    for h, s in zip(hist, stats):
        assert s["converged"]
        assert abs(s["c"] - h["c"]) <= 1e-8 * h["c"]
        assert abs(s["lambda"] - h["lam"]) <= 1e-7 * h["lam"]
        assert abs(s["change"] - h["change"]) <= 1e-7
        assert abs(s["volume"] - h["volume"]) <= 1e-8 * h["volume"]
    np.testing.assert_allclose(xg, xo, atol=1e-7)


@pytest.mark.parametrize("mode", ["density", "sensitivity"])
def test_iterate_matches_oracle_with_passive_elements(mode):
    p = ragged_problem(30, (16, 8, 6), rmin=2.0)
    p.f = np.zeros(p.ndof)
    p.f[3 * int(p.node_id(16, 0, 3)) + 1] = -1.0
    p.mask[p.mask == 2] = 0
    p.filter_mode = mode
    n = 6
    xo, hist = simp.SimpOracle(p).trajectory(n)
    xg, stats = run_gpu_trajectory(p, n)
    for h, s in zip(hist, stats):
        assert abs(s["c"] - h["c"]) <= 1e-8 * h["c"], (s["c"], h["c"])
    np.testing.assert_allclose(xg, xo, atol=1e-7)
    assert np.all(xg[p.mask == 1] == 0.0)


def test_iterate_matches_oracle_with_volume_over_all_elements():
    """vol_mode "all" with fixed-solid and fixed-void elements: the trajectory
    matches the oracle's, and the physical density summed over every element
    meets volfrac * nel."""
    p = ragged_problem(31, (16, 8, 6), rmin=2.0)
    p.f = np.zeros(p.ndof)
    p.f[3 * int(p.node_id(16, 0, 3)) + 1] = -1.0
    p.vol_mode = "all"
    assert (p.mask == 2).sum() > 0
    n = 4
    o = simp.SimpOracle(p)
    xo, hist = o.trajectory(n)
    xg, stats = run_gpu_trajectory(p, n)
    for h, s in zip(hist, stats):
        assert abs(s["c"] - h["c"]) <= 1e-8 * h["c"], (s["c"], h["c"])
    np.testing.assert_allclose(xg, xo, atol=1e-7)
    assert abs(o.physical(xg).sum() - p.volfrac * p.nel) <= 1e-7 * p.nel


@pytest.mark.parametrize("warm", [0, 1, 2, 3])
def test_warm_start_modes_give_the_same_trajectory(warm):
    """Zero, last, extrapolated and energy-projected initial guesses change only
    the CG iteration counts: the trajectory matches the oracle's (direct
    solves) to the solve tolerance."""
    p = synth.config_small()
    n_iter = 6
    ref = simp.SimpOracle(p).trajectory(n_iter)[1]
    with topo.Context(p, topo.default_opts(rtol=1e-10, warm_start=warm)) as ctx:
        x = dev(p.initial_design())
        st = ctx.iterate(x, n_iter)
    for k in range(n_iter):
        assert abs(st[k]["c"] - ref[k]["c"]) <= 1e-8 * abs(ref[k]["c"]), (warm, k)
    print("warm", warm, "iterations", [s["pcg_iters"] for s in st])


@functools.lru_cache(maxsize=1)
def _lagged_case():
    p = synth.cantilever(24, 12, 12, volfrac=0.3, rmin=1.5, n_iter=6)
    return p, simp.SimpOracle(p).trajectory(6)[1]


@pytest.mark.parametrize("refresh", [1, 3])
def test_lagged_coarse_inverse_gives_the_same_trajectory(refresh):
    """A coarse inverse kept over several SIMP iterations only changes the CG
    iteration counts (24x12x12: 3 levels, a coarsest level of 336 dofs); the
    compliances match the oracle's direct solves to the solve tolerance."""
    p, ref = _lagged_case()
    n_iter = len(ref)
    with topo.Context(p, topo.default_opts(rtol=1e-10, coarse_refresh=refresh)) as ctx:
        assert ctx.mg_levels == 3
        x = dev(p.initial_design())
        st = ctx.iterate(x, n_iter)
    for k in range(n_iter):
        assert abs(st[k]["c"] - ref[k]["c"]) <= 1e-8 * abs(ref[k]["c"]), (refresh, k)
    print("refresh", refresh, "iterations", [s["pcg_iters"] for s in st])
