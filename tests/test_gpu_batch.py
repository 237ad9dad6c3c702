"""Batched SIMP iterations: every problem of a batch ends exactly where its own
single-problem run ends (same kernels, same order on its own stream), and the
launch-shape autotuner changes nothing but rounding."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu


def problems():
    out = []
    for seed, nelx in [(0, 24), (1, 32), (2, 16), (3, 40), (4, 24), (5, 16)]:
        out.append(synth.random_problem(seed, nelx, n_iter=4))
    return out


def run_single(p, opts, n_iter):
    with topo.Context(p, opts) as ctx:
        x = torch.from_numpy(p.initial_design()).to("cuda")
        st = ctx.iterate(x, n_iter)
        torch.cuda.synchronize()
        return x.cpu().numpy(), [s["c"] for s in st]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_problem_runs(precision):
    ps = problems()
    opts = topo.default_opts(precision=topo.PREC_FP64 if precision == "fp64" else topo.PREC_FP32)
    n_iter = 4
    with topo.Batch(ps, opts, n_threads=4) as b:
        xs = [torch.from_numpy(p.initial_design()).to("cuda") for p in ps]
        stats = b.iterate(xs, n_iter)
        torch.cuda.synchronize()
        got = [x.cpu().numpy() for x in xs]
    for i, p in enumerate(ps):
        xr, cr = run_single(p, opts, n_iter)
        assert np.array_equal(got[i], xr), i
        assert [s["c"] for s in stats[i]] == cr, i


def test_autotuned_shapes_change_only_rounding():
    """Other launch shapes change reduction orders, hence the CG iterates at the
    rounding level; solving to 1e-12 keeps the trajectories within 1e-9."""
    ps = problems()[:3]
    n_iter = 3
    base = [run_single(p, topo.default_opts(rtol=1e-12), n_iter) for p in ps]
    with topo.Batch(ps, topo.default_opts(autotune=1, rtol=1e-12), n_threads=3) as b:
        xs = [torch.from_numpy(p.initial_design()).to("cuda") for p in ps]
        stats = b.iterate(xs, n_iter)
        torch.cuda.synchronize()
        for i in range(len(ps)):
            c = np.array([s["c"] for s in stats[i]])
            cr = np.array(base[i][1])
            assert np.abs(c - cr).max() <= 1e-9 * np.abs(cr).max(), i
            assert np.abs(xs[i].cpu().numpy() - base[i][0]).max() <= 1e-7, i


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grouped_launches_equal_separate_streams(precision):
    """Ten problems on one grid (a group of 8 and one of 2) plus two of another
    size: with grouped launches every problem ends bit for bit where it ends on
    its own stream (group_launch 0); the CG iteration counts agree too."""
    ps = [synth.random_problem(100 + s, 16, n_iter=3) for s in range(10)]
    ps += [synth.random_problem(200 + s, 24, n_iter=3) for s in range(2)]
    prec = topo.PREC_FP64 if precision == "fp64" else topo.PREC_FP32
    res = {}
    for grouped in (0, 1):
        with topo.Batch(ps, topo.default_opts(precision=prec, group_launch=grouped), n_threads=4) as b:
            xs = [torch.from_numpy(p.initial_design()).to("cuda") for p in ps]
            st = b.iterate(xs, 3)
            torch.cuda.synchronize()
            res[grouped] = ([x.cpu().numpy() for x in xs], st)
    for i in range(len(ps)):
        assert np.array_equal(res[0][0][i], res[1][0][i]), i
        assert [s["c"] for s in res[0][1][i]] == [s["c"] for s in res[1][1][i]], i
        assert [s["pcg_iters"] for s in res[0][1][i]] == [s["pcg_iters"] for s in res[1][1][i]], i
        assert [s["volume"] for s in res[0][1][i]] == [s["volume"] for s in res[1][1][i]], i


def test_grouped_launches_equal_separate_streams_on_a_large_grid():
    """Two problems of 101x71x69 elements (large enough for the per-cell
    prolongation on the finest level): grouped launches end bit for bit where
    separate streams do."""
    ps = [synth.cantilever(101, 71, 69, volfrac=v, rmin=1.5, n_iter=2) for v in (0.3, 0.2)]
    res = {}
    for grouped in (0, 1):
        with topo.Batch(ps, topo.default_opts(precision=topo.PREC_FP32, group_launch=grouped), n_threads=2) as b:
            xs = [torch.from_numpy(p.initial_design()).to("cuda") for p in ps]
            st = b.iterate(xs, 2)
            torch.cuda.synchronize()
            res[grouped] = ([x.cpu().numpy() for x in xs], st)
    for i in range(len(ps)):
        assert np.array_equal(res[0][0][i], res[1][0][i]), i
        assert [s["pcg_iters"] for s in res[0][1][i]] == [s["pcg_iters"] for s in res[1][1][i]], i


@pytest.mark.parametrize("variant", ["extrapolated-sens", "zero-keep-inverse", "last-mixed-reach"])
def test_grouped_iterations_cover_every_warm_start_and_filter(variant):
    """Grouped SIMP phases (filter, operator set-up and coarse inverse, warm
    starts, sensitivities, OC) against per-problem streams, bit for bit, under
    the other warm starts, the sensitivity filter, a coarse inverse kept for two
    iterations and stencils of different reach within one group."""
    ps = [synth.random_problem(300 + s, 16, n_iter=4) for s in range(5)]
    kw = dict(precision=topo.PREC_FP32)
    if variant == "extrapolated-sens":
        kw["warm_start"] = 2
        for p in ps:
            p.filter_mode = "sensitivity"
    elif variant == "zero-keep-inverse":
        kw.update(warm_start=0, coarse_refresh=2, precision=topo.PREC_FP64)
    else:
        kw["warm_start"] = 1
        for k, p in enumerate(ps):
            p.rmin = [1.5, 2.5, 3.5, 1.8, 4.5][k]  # reaches 1, 2, 3, 1 and the offset-list kernel
    res = {}
    for grouped in (0, 1):
        with topo.Batch(ps, topo.default_opts(group_launch=grouped, **kw), n_threads=2) as b:
            xs = [torch.from_numpy(p.initial_design()).to("cuda") for p in ps]
            st = b.iterate(xs, 4)
            torch.cuda.synchronize()
            res[grouped] = ([x.cpu().numpy() for x in xs], st)
    for i in range(len(ps)):
        assert np.array_equal(res[0][0][i], res[1][0][i]), i
        for key in ("c", "pcg_iters", "volume", "change", "lambda"):
            assert [s[key] for s in res[0][1][i]] == [s[key] for s in res[1][1][i]], (i, key)


def test_autotuner_remembers_shapes_per_grid():
    """After the cache is cleared, the first context on a grid times the launch
    shapes; a second context on the same grid takes the remembered shapes, so
    the two runs agree bit for bit (fresh timings could pick other shapes,
    which would change the rounding)."""
    lib = topo.load()
    lib.topo_clear_tuning_cache()
    p = synth.random_problem(7, 32, n_iter=3)
    opts = topo.default_opts(precision=topo.PREC_FP32, autotune=1)
    a = run_single(p, opts, 3)
    b = run_single(p, opts, 3)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    lib.topo_clear_tuning_cache()
