"""Single-precision multigrid preconditioner inside FP64 flexible CG: the
solution meets the same FP64 residual tolerance, and the SIMP trajectory stays
within stated bounds of the FP64 one.  Variants: FP32 on the vector units (both
K.u kernels, the element-column one also with its LDS-staged shapes), FP32 on
the matrix cores (mfma_smoothing), BF16 operands on the matrix cores."""

import numpy as np
import pytest

import synth
from oracle import fem, mg
from oracle.ke import element_stiffness

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu
KE = element_stiffness(0.3)


VARIANTS = {
    "fp32": dict(precision=topo.PREC_FP32),
    # every level and the CG product on the element-column shapes whose node
    # planes are staged through LDS (the finest-level default on large grids)
    "fp32_staged": dict(precision=topo.PREC_FP32, ku_shape=13),
    "fp32_staged16": dict(precision=topo.PREC_FP32, ku_shape=14),
    # per-level smoother degrees, finest first (the benchmark's setting)
    "fp32_levels": dict(precision=topo.PREC_FP32, cheb_degree_level=[1, 2, 4, 6]),
    "fp32_node": dict(precision=topo.PREC_FP32, ku_kernel=topo.KU_NODE),
    "fp32_mfma": dict(precision=topo.PREC_FP32, mfma_smoothing=1),
    "bf16": dict(precision=topo.PREC_BF16),
}


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("case", ["small", "obstacle"])
def test_low_precision_preconditioned_solve_meets_fp64_tolerance(case, variant):
    p = synth.config_small() if case == "small" else synth.config_obstacle(seed=4)
    x = synth.random_density(3, p.nel, 0.05, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    f = p.f.copy()
    f[p.fixed_dofs] = 0.0
    edof = fem.element_dofs(p.nelx, p.nely, p.nelz)
    out = {}
    for name, kw in (("fp64", {}), (variant, VARIANTS[variant])):
        with topo.Context(p, topo.default_opts(rtol=1e-10, max_iters=3000, **kw)) as ctx:
            u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
            st = ctx.solve(torch.from_numpy(x).cuda(), u)
            out[name] = (u.cpu().numpy(), st)
    for name, (u, st) in out.items():
        assert st["converged"]
        # true FP64 residual of the returned solution, by the oracle's operator
        res = f - fem.apply_K_reduced(E, KE, edof, u, p.fixed_dofs)
        assert np.linalg.norm(res) <= 3e-10 * np.linalg.norm(f), name
    u64, ul = out["fp64"][0], out[variant][0]
    assert abs(f @ ul - f @ u64) <= 1e-9 * abs(f @ u64)
    # a single-precision preconditioner costs at most a few extra iterations; BF16
    # operands (relative rounding 2^-9 in the smoother) up to a quarter more
    extra = 5 if variant != "bf16" else max(5, out["fp64"][1]["iters"] // 4)
    print(variant, "iterations", out[variant][1]["iters"], "fp64", out["fp64"][1]["iters"])
    assert out[variant][1]["iters"] <= out["fp64"][1]["iters"] + extra


@pytest.mark.parametrize("cap", [140, 1500])
@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("case", ["small", "ragged"])
def test_low_precision_preconditioner_matches_oracle(case, variant, cap):
    """One V-cycle application against the oracle's FP64 V-cycle: FP32 arithmetic
    (2^-24 rounding through a few dozen passes) within 1e-4 of the output scale;
    BF16 operands in the smoothing products (2^-9) within 3e-2."""
    if case == "small":
        p = synth.config_small()
    else:
        p = synth.cantilever(13, 7, 5, volfrac=0.3, rmin=2.0, n_iter=5)
    x = synth.random_density(5, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    fm = np.zeros(p.ndof, bool)
    fm[p.fixed_dofs] = True
    r = synth.random_vector(6, p.ndof)
    r[fm] = 0.0
    # the default smoother degrees: one step on the finest level, four below
    ref = mg.VCycle(p, E, KE, degree=1, coarse_degree=4, max_coarse_dof=cap,
                    level_degrees=VARIANTS[variant].get("cheb_degree_level")).apply(r)
    with topo.Context(p, topo.default_opts(mg_max_coarse_dof=cap, cheb_degree=1, cheb_degree_coarse=4,
                                           **VARIANTS[variant])) as ctx:
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(torch.from_numpy(x).cuda(), torch.from_numpy(r).cuda(), z)
        torch.cuda.synchronize()
        got = z.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(variant, case, cap, "max rel err", err)
    assert err <= (3e-2 if variant == "bf16" else 1e-4)


@pytest.mark.parametrize("variant", ["fp32", "fp32_levels", "bf16"])
def test_low_precision_preconditioner_on_five_levels_matches_oracle(variant):
    """33x17x17 at a 140-dof cap: 5 levels, so the per-level degrees 1, 2, 4, 6
    each smooth a level of their own."""
    p = synth.cantilever(33, 17, 17, volfrac=0.3, rmin=1.5, n_iter=1)
    x = synth.random_density(5, p.nel, 0.0, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    fm = np.zeros(p.ndof, bool)
    fm[p.fixed_dofs] = True
    r = synth.random_vector(6, p.ndof)
    r[fm] = 0.0
    lev = VARIANTS[variant].get("cheb_degree_level")
    V = mg.VCycle(p, E, KE, degree=1, coarse_degree=4, max_coarse_dof=140, level_degrees=lev)
    assert len(V.levels) == 5
    ref = V.apply(r)
    with topo.Context(p, topo.default_opts(mg_max_coarse_dof=140, cheb_degree=1, cheb_degree_coarse=4,
                                           **VARIANTS[variant])) as ctx:
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(torch.from_numpy(x).cuda(), torch.from_numpy(r).cuda(), z)
        torch.cuda.synchronize()
        got = z.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(variant, "5 levels, max rel err", err)
    assert err <= (3e-2 if variant == "bf16" else 1e-4)


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_low_precision_preconditioner_trajectory_close_to_fp64(variant):
    """The preconditioner does not change the solution beyond the solve tolerance
    (1e-10), so the SIMP trajectories agree to about that level."""
    p = synth.config_small()
    res = {}
    for name, kw in (("fp64", {}), (variant, VARIANTS[variant])):
        with topo.Context(p, topo.default_opts(rtol=1e-10, **kw)) as ctx:
            x = torch.from_numpy(p.initial_design()).cuda()
            stats = ctx.iterate(x, p.n_iter)
            res[name] = (x.cpu().numpy(), [s["c"] for s in stats])
    c64, cl = np.array(res["fp64"][1]), np.array(res[variant][1])
    assert np.max(np.abs(cl - c64) / c64) <= 1e-8
    assert np.abs(res[variant][0] - res["fp64"][0]).max() <= 1e-6
