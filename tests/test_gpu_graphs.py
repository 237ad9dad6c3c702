"""Graph replay versus direct launches, chunked convergence checks, and
determinism of the GPU path (same inputs -> bitwise identical outputs)."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu


def trajectory(p, n, **opt):
    with topo.Context(p, topo.default_opts(rtol=1e-10, **opt)) as ctx:
        x = torch.from_numpy(p.initial_design()).to("cuda")
        stats = ctx.iterate(x, n)
        torch.cuda.synchronize()
        return x.cpu().numpy(), stats


def test_graph_replay_equals_direct_launches():
    p = synth.config_small()
    xg, sg = trajectory(p, 4, use_graphs=1, check_every=4)
    xd, sd = trajectory(p, 4, use_graphs=0, check_every=4)
    assert np.array_equal(xg, xd)
    assert [s["c"] for s in sg] == [s["c"] for s in sd]
    assert [s["pcg_iters"] for s in sg] == [s["pcg_iters"] for s in sd]


@pytest.mark.parametrize("chunk", [1, 3, 8])
def test_chunked_checks_stop_at_the_same_iteration(chunk):
    """The device stops iterating at convergence inside a chunk, so the iteration
    count and the result do not depend on how often the host looks."""
    p = synth.config_small()
    x1, s1 = trajectory(p, 3, check_every=1, use_graphs=0)
    xc, sc = trajectory(p, 3, check_every=chunk, use_graphs=1)
    assert [s["pcg_iters"] for s in s1] == [s["pcg_iters"] for s in sc]
    assert np.array_equal(x1, xc)


def test_repeated_runs_are_bitwise_identical():
    p = synth.config_obstacle(seed=2)
    p.n_iter = 2
    a, sa = trajectory(p, 2)
    b, sb = trajectory(p, 2)
    assert np.array_equal(a, b)
    assert [s["c"] for s in sa] == [s["c"] for s in sb]


def test_solve_reports_nonconvergence():
    p = synth.config_small()
    with topo.Context(p, topo.default_opts(max_iters=2, rtol=1e-12)) as ctx:
        x = torch.full((p.nel,), 0.3, dtype=torch.float64, device="cuda")
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        st = ctx.solve(x, u, raise_on_nonconv=False)
        assert not st["converged"] and st["iters"] == 2
        with pytest.raises(topo.NotConverged):
            ctx.solve(x, torch.zeros_like(u))


@pytest.mark.parametrize("graphs", [0, 1])
def test_chunks_enqueued_past_convergence_change_nothing(graphs):
    """A long solve makes the next one enqueue several chunks before its first
    host check; a solve that converges well inside them (from a close initial
    guess) ends where a fresh context's does, bit for bit, with the same count."""
    p = synth.config_small()
    x = torch.from_numpy(synth.random_density(3, p.nel, 0.05, 1.0)).to("cuda")
    opts = topo.default_opts(rtol=1e-12, check_every=2, use_graphs=graphs)
    with topo.Context(p, opts) as ctx:
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        long = ctx.solve(x, u)
        guess = u * (1.0 + 1e-9 * torch.from_numpy(synth.random_vector(4, p.ndof)).to("cuda"))
        u2 = guess.clone()
        short = ctx.solve(x, u2)
    print("iterations", long["iters"], short["iters"])
    # the first check of the second solve comes after 3/5 of the first one's
    # iterations, past its convergence
    assert 3 * long["iters"] // 5 >= short["iters"] + 2 >= 3
    with topo.Context(p, opts) as fresh:
        u3 = guess.clone()
        ref = fresh.solve(x, u3)
    assert short["iters"] == ref["iters"]
    assert torch.equal(u2, u3)
