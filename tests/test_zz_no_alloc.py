"""The allocation-free OC entry point (topo_oc_update_noalloc) against the
context entry point topo_oc_update: two calls in a row, the second on a smaller
problem, each compared with the context's result on the same inputs."""

import numpy as np
import pytest

import synth
from oracle import filt

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda")


def oc_inputs(seed, dims, rmin):
    q = synth.cantilever(*dims, volfrac=0.3, rmin=rmin, n_iter=1)
    rng = np.random.default_rng(seed)
    m = np.zeros(q.nel, np.int8)
    m[rng.random(q.nel) < 0.08] = 1
    m[rng.random(q.nel) < 0.03] = 2
    q.mask = m
    F = filt.Filter(*dims, rmin, m)
    design = m == 0
    x = q.initial_design()
    x[design] = rng.uniform(0.0, 2 * q.volfrac, design.sum())
    dc = F.adjoint(-rng.exponential(1.0, q.nel) * 10 ** rng.uniform(-3, 2))
    return q, x, dc, F.volume_weights()


def test_noalloc_oc_update_matches_context_entry_point():
    for seed, dims in ((0, (41, 23, 17)), (1, (13, 7, 5))):  # the second call is smaller
        q, x, dc, w = oc_inputs(seed, dims, 2.0)
        target = q.volfrac * int((q.mask == 0).sum())
        with topo.Context(q) as ctx:
            xn_ref = torch.empty(q.nel, dtype=torch.float64, device="cuda")
            chg_ref, lam_ref = ctx.oc_update(dev(x), dev(dc), dev(w), xn_ref)
            ref = xn_ref.cpu().numpy()
        xn = torch.full((q.nel,), -1.0, dtype=torch.float64, device="cuda")
        res = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
        topo.oc_update_noalloc(dev(x), dev(dc), dev(w), dev(q.mask, np.int8), q.move, q.eta, target, 1e-12,
                               xn, res)
        torch.cuda.synchronize()
        got = xn.cpu().numpy()
        chg, vol, lam = res.cpu().numpy()
        # same kernels, same order of summation: the same bits
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert chg == chg_ref and lam == lam_ref, (chg, chg_ref, lam, lam_ref)
        assert abs(vol - w @ got) <= 1e-12 * abs(vol)
        print(f"noalloc OC {dims}: lambda {lam:.6e}, change {chg:.4f}")
