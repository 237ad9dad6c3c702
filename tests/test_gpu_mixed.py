"""Single-precision multigrid preconditioner inside FP64 flexible CG: the
solution meets the same FP64 residual tolerance, and the SIMP trajectory stays
within stated bounds of the FP64 one."""

import numpy as np
import pytest

import synth
from oracle import fem, mg
from oracle.ke import element_stiffness

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu
KE = element_stiffness(0.3)


@pytest.mark.parametrize("case", ["small", "obstacle"])
def test_fp32_preconditioned_solve_meets_fp64_tolerance(case):
    p = synth.config_small() if case == "small" else synth.config_obstacle(seed=4)
    x = synth.random_density(3, p.nel, 0.05, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    f = p.f.copy()
    f[p.fixed_dofs] = 0.0
    edof = fem.element_dofs(p.nelx, p.nely, p.nelz)
    out = {}
    for prec in (topo.PREC_FP64, topo.PREC_FP32):
        with topo.Context(p, topo.default_opts(precision=prec, rtol=1e-10, max_iters=3000)) as ctx:
            u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
            st = ctx.solve(torch.from_numpy(x).cuda(), u)
            out[prec] = (u.cpu().numpy(), st)
    for prec, (u, st) in out.items():
        assert st["converged"]
        # true FP64 residual of the returned solution, by the oracle's operator
        res = f - fem.apply_K_reduced(E, KE, edof, u, p.fixed_dofs)
        assert np.linalg.norm(res) <= 3e-10 * np.linalg.norm(f), prec
    u64, u32 = out[topo.PREC_FP64][0], out[topo.PREC_FP32][0]
    assert abs(f @ u32 - f @ u64) <= 1e-9 * abs(f @ u64)
    # the preconditioner in single precision costs at most a few extra iterations
    assert out[topo.PREC_FP32][1]["iters"] <= out[topo.PREC_FP64][1]["iters"] + 5


def test_fp32_preconditioner_trajectory_close_to_fp64():
    p = synth.config_small()
    res = {}
    for prec in (topo.PREC_FP64, topo.PREC_FP32):
        with topo.Context(p, topo.default_opts(precision=prec, rtol=1e-10)) as ctx:
            x = torch.from_numpy(p.initial_design()).cuda()
            stats = ctx.iterate(x, p.n_iter)
            res[prec] = (x.cpu().numpy(), [s["c"] for s in stats])
    c64, c32 = np.array(res[topo.PREC_FP64][1]), np.array(res[topo.PREC_FP32][1])
    assert np.max(np.abs(c32 - c64) / c64) <= 1e-8
    assert np.abs(res[topo.PREC_FP32][0] - res[topo.PREC_FP64][0]).max() <= 1e-6


def test_bf16_reports_unsupported():
    p = synth.config_small()
    with pytest.raises(topo.TopoError) as e:
        topo.Context(p, topo.default_opts(precision=topo.PREC_BF16))
    assert e.value.status == 5
