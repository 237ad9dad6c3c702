#!/usr/bin/env python3
"""Benchmark of the SIMP hot path on one MI355X.

Workload: the 160x80x80 cantilever (1,024,000 hexahedra, 3,168,963 DOF; face x=0
clamped, unit downward load spread over the bottom edge of the free end),
volfrac 0.2, rmin 3.0, p = 3, density filter, CG to an FP64 relative residual
of 1e-8 with warm starts, preconditioned by a multigrid V-cycle in FP32 (FP64
with --precision fp64); a lockstep FP64 run reports the mixed path's compliance
and displacement error.  A step is one full SIMP iteration (filter, moduli and
multigrid set-up, solve, sensitivities, filter adjoint, OC update).  Prints one
JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/SIMP iter @3.1M DOF; PCG iters+time to 1e-8 rel res, learned vs plain MG"
HBM_PEAK_GBS = 8000.0             # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ku_element_fp64_160x80x80_traffic.json")


def ku_algorithmic_bytes(p):
    """Bytes a K.u launch (y = K u) must move: u read and y written
    (8 B per dof each), the element moduli read (8 B per element) and the
    fixed-dof flags read (1 B per node)."""
    nnodes = (p.nelx + 1) * (p.nely + 1) * (p.nelz + 1)
    return 2 * 8 * p.ndof + 8 * p.nel + nnodes


def ku_traffic_bytes():
    """HBM bytes per K.u launch from the committed counter runs (FETCH_SIZE and
    WRITE_SIZE scaled by what the same counters read for a copy kernel of known
    size), if they were taken on the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for src in rec.get("kernel_sources", []):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if rec.get("kernel_source_sha256") != h.hexdigest():
        return None
    return rec.get("bytes_per_launch")


ORACLE_ITER_FILE = os.path.join(ROOT, "profiles", "cpu_oracle_simp_iteration_160x80x80.json")
ORACLE_SOURCES = ["oracle/ke.py", "oracle/fem.py", "oracle/filt.py", "oracle/mg.py", "oracle/oc.py",
                  "oracle/simp.py"]


def _sources_sha256(paths):
    h = hashlib.sha256()
    for src in paths:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _host_cpu():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def oracle_full_iteration(p, rtol=1e-8, n_iter=4):
    """Complete SIMP iterations of the oracle at the benchmark grid from the
    initial design, each timed by phase: physical density (filter), moduli,
    assembly of the multigrid hierarchy (fine operator included), CG
    preconditioned by the oracle's V-cycle from zero to rtol, energies and
    sensitivities, filter adjoint and the exact OC multiplier.  The filter matrix
    and the element dof map are per-problem set-up (the GPU's set-up is not
    timed either) and are reported apart.  iteration_s is the mean over the
    iterations after the first (the first, on a uniform design, solves in fewer
    CG iterations than the later ones)."""
    import numpy as np
    from oracle import simp

    t0 = time.perf_counter()
    so = simp.SimpOracle(p)
    setup = time.perf_counter() - t0
    fm = np.zeros(p.ndof, bool)
    fm[p.fixed_dofs] = True
    f = p.f.copy()
    f[fm] = 0.0
    x = p.initial_design()
    its = []
    for k in range(n_iter):
        rec, x = _oracle_timed_step(p, so, f, x, rtol)
        its.append(rec)
        print(f"# oracle SIMP iteration {k + 1}: {rec['iteration_s']:.1f} s, {rec['pcg_iters']} CG iterations",
              file=sys.stderr, flush=True)
    later = its[1:] if len(its) > 1 else its
    return {"iteration_s": float(np.mean([r["iteration_s"] for r in later])),
            "iterations": its, "setup_filter_and_dofs_s": round(setup, 3),
            "pcg_iters_mean": float(np.mean([r["pcg_iters"] for r in later])),
            "mg_levels": its[0]["mg_levels"], "blas_threads": _blas_threads()}


def _oracle_timed_step(p, so, f, x, rtol):
    from oracle import fem, mg, oc

    t = {}
    t0 = time.perf_counter()
    xphys = so.physical(x)
    E = fem.simp_modulus(xphys, p.E0, p.Emin, p.penal)
    t["filter_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    V = mg.VCycle(p, E, so.KE, degree=2, max_coarse_dof=1500)
    t["assembly_and_mg_setup_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    u, iters, relres = mg.pcg(V.levels[0].A, f, V.apply, rtol=rtol, max_iter=1000)
    t["pcg_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ce = fem.element_energy(so.KE, so.edof, u)
    c = fem.compliance(f, u)
    dc = fem.compliance_sensitivity(xphys, ce, p.E0, p.Emin, p.penal)
    t["sensitivity_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    dcf = so.filter.adjoint(dc)
    t["filter_s"] += time.perf_counter() - t0
    t0 = time.perf_counter()
    xnew, lam = oc.oc_exact(x, dcf, so.w, so.w, so.target, p.move, p.eta, so.design)
    t["oc_s"] = time.perf_counter() - t0
    return ({"iteration_s": round(sum(t.values()), 3), "phases": {k: round(v, 3) for k, v in t.items()},
             "pcg_iters": int(iters), "relres": relres, "compliance": c, "mg_levels": len(V.levels)}, xnew)


def record_oracle_iteration(p):
    """Runs oracle_full_iteration once and writes its record (with the host's
    processor and the oracle sources' hash) next to the kernel profiles."""
    rec = oracle_full_iteration(p)
    rec.update(workload=p.name, command="python bench.py --record-oracle-iteration", host=_host_cpu(),
               oracle_sources=ORACLE_SOURCES, oracle_source_sha256=_sources_sha256(ORACLE_SOURCES),
               solver="CG from zero to 1e-8, preconditioned by the oracle's V-cycle (Chebyshev degree 2, "
                      "coarsest level <= 1500 dofs, dense Cholesky); SciPy sparse products are single-threaded")
    os.makedirs(os.path.dirname(ORACLE_ITER_FILE), exist_ok=True)
    with open(ORACLE_ITER_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def recorded_oracle_iteration():
    """The recorded full oracle iteration, if it was taken with the current
    oracle sources (else None)."""
    if not os.path.exists(ORACLE_ITER_FILE):
        return None
    with open(ORACLE_ITER_FILE) as fh:
        rec = json.load(fh)
    if rec.get("oracle_source_sha256") != _sources_sha256(rec.get("oracle_sources", [])):
        return None
    return rec


def oracle_live_sample(p):
    """The oracle's non-solve phases of one SIMP iteration at the benchmark grid,
    timed live: physical density, energies and sensitivities, filter adjoint and
    the exact OC multiplier (the filter matrix is built first, untimed)."""
    import numpy as np
    from oracle import fem, oc, simp

    so = simp.SimpOracle(p)
    rng = np.random.default_rng(0)
    x = p.initial_design()
    u = rng.standard_normal(p.ndof) * 1e-2
    u[p.fixed_dofs] = 0.0
    t0 = time.perf_counter()
    xphys = so.physical(x)
    t1 = time.perf_counter()
    ce = fem.element_energy(so.KE, so.edof, u)
    dc = fem.compliance_sensitivity(xphys, ce, p.E0, p.Emin, p.penal)
    t2 = time.perf_counter()
    dcf = so.filter.adjoint(dc)
    t3 = time.perf_counter()
    oc.oc_exact(x, dcf, so.w, so.w, so.target, p.move, p.eta, so.design)
    t4 = time.perf_counter()
    return {"filter_s": round((t1 - t0) + (t3 - t2), 3), "sensitivity_s": round(t2 - t1, 3),
            "oc_s": round(t4 - t3, 3)}


def cpu_baseline(p, ku_equiv_per_iter, budget_s):
    """The oracle on the host cores.  value: one complete oracle SIMP iteration at
    the benchmark grid as recorded by --record-oracle-iteration (its solve alone
    takes minutes), valid while the oracle sources are unchanged; the non-solve
    phases are re-timed live in this run beside the recorded ones.  Without a
    valid record: a model (one live oracle K.u scaled by the K.u applications of
    the GPU's iteration), labelled as such."""
    import numpy as np
    from oracle import fem
    from oracle.ke import element_stiffness

    rec = recorded_oracle_iteration()
    live = oracle_live_sample(p)
    if rec is not None:
        ph = {k: round(float(sum(it["phases"][k] for it in rec["iterations"][1:]) /
                             max(1, len(rec["iterations"]) - 1)), 3) for k in rec["iterations"][0]["phases"]}
        return {
            "value": round(1e3 * rec["iteration_s"], 1), "unit": "ms/SIMP iteration", "cores": 1,
            "kind": "oracle",
            "sample": (f"complete oracle SIMP iterations at 160x80x80 (filter, assembly and multigrid set-up, "
                       f"CG from zero to 1e-8, {rec['pcg_iters_mean']:.1f} iterations on average, sensitivities, "
                       f"filter adjoint, exact OC multiplier): the mean of iterations 2-{len(rec['iterations'])} "
                       f"of the oracle's own trajectory, recorded by "
                       f"`{rec['command']}` on {rec['host']['model']} ({rec['host']['nproc']} cores; SciPy's "
                       f"sparse products are single-threaded, so one core did the work); its filter, "
                       f"sensitivity and OC phases re-timed live in this run"),
            "phases_recorded_s": ph, "phases_live_s": live,
            "host_live": _host_cpu(),
        }
    KE = element_stiffness(p.nu)
    edof = fem.element_dofs(p.nelx, p.nely, p.nelz)
    rng = np.random.default_rng(0)
    E = fem.simp_modulus(rng.uniform(0, 1, p.nel), p.E0, p.Emin, p.penal)
    u = rng.standard_normal(p.ndof)
    t0 = time.perf_counter()
    reps = 0
    while True:
        fem.apply_K(E, KE, edof, u)
        reps += 1
        if time.perf_counter() - t0 > min(budget_s, 10.0) or reps >= 3:
            break
    t_ku = (time.perf_counter() - t0) / reps
    ms_iter = 1e3 * (t_ku * ku_equiv_per_iter + sum(live.values()))
    return {
        "value": round(ms_iter, 1), "unit": "ms/SIMP iteration", "cores": int(_blas_threads()),
        "kind": "model",
        "sample": (f"no valid recorded oracle iteration: oracle element-by-element K.u at 160x80x80 "
                   f"({t_ku:.2f} s/call, {reps} calls) scaled by the {ku_equiv_per_iter:.1f} fine-grid "
                   f"K.u-equivalents of the GPU's SIMP iteration, plus the live non-solve phases"),
        "phases_live_s": live,
    }


PAPER_TABLE = {  # the paper's Performance Comparison table, PyTopo3D column (seconds, 200 iterations)
    "hardware": "Intel Core Ultra 7 155U laptop CPU", "assembly_s": 33.9, "solve_s": 99.8,
    "filter_s": 0.7, "update_s": 10.8, "total_s": 147.3}


def paper_benchmark(topo, synth, args):
    """The paper's own timed workload (32x16x16 cantilever, point load, volfrac 0.2,
    p 3, rmin 4.0: 251-point filter, 200 OC iterations) on the GPU path, with the
    phase split of the paper's table (assembly has no counterpart here: the
    operator is matrix-free, its set-up is inside the solve phase)."""
    import torch

    p = synth.config_paper_benchmark()
    with topo.Context(p, topo.default_opts(rtol=1e-8)) as ctx:
        x = torch.from_numpy(p.initial_design()).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.iterate(x, p.n_iter, raise_on_nonconv=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    tot = {k: sum(r[k] for r in st) * 1e-3 for k in ("ms_filter", "ms_solve", "ms_sens", "ms_oc")}
    print(f"# paper benchmark: {p.n_iter} iterations in {wall:.2f} s", file=sys.stderr, flush=True)
    return {
        "workload": "32x16x16 cantilever (28,611 DOF), point load, volfrac 0.2, p 3, rmin 4.0, 200 iterations",
        "total_s": round(wall, 3), "solve_s": round(tot["ms_solve"], 3),
        "filter_s": round(tot["ms_filter"], 3), "sensitivity_s": round(tot["ms_sens"], 3),
        "update_s": round(tot["ms_oc"], 3),
        "pcg_iters_mean": round(sum(r["pcg_iters"] for r in st) / len(st), 2),
        "compliance_final": st[-1]["c"],
        "paper_table": PAPER_TABLE,
    }


def paper_benchmark_oracle(budget_s):
    """The oracle's SIMP iteration on the paper's workload (direct solve), timed by
    phase on a few iterations and scaled to 200."""
    import numpy as np
    import synth
    from oracle import fem, oc, simp

    p = synth.config_paper_benchmark()
    so = simp.SimpOracle(p)
    x = p.initial_design()
    ph = {"solve": 0.0, "filter": 0.0, "update": 0.0}
    n = 0
    t_start = time.perf_counter()
    while n < 2 and (n == 0 or time.perf_counter() - t_start < budget_s):
        t0 = time.perf_counter()
        xphys = so.physical(x)
        t1 = time.perf_counter()
        E = fem.simp_modulus(xphys, p.E0, p.Emin, p.penal)
        u = so.solve(E)
        t2 = time.perf_counter()
        ce = fem.element_energy(so.KE, so.edof, u)
        dc = fem.compliance_sensitivity(xphys, ce, p.E0, p.Emin, p.penal)
        dcf = so.filter.adjoint(dc)
        t3 = time.perf_counter()
        x, _ = oc.oc_exact(x, dcf, so.w.copy(), so.w, so.target, p.move, p.eta, so.design)
        t4 = time.perf_counter()
        ph["filter"] += (t1 - t0) + (t3 - t2)
        ph["solve"] += t2 - t1
        ph["update"] += t4 - t3
        n += 1
    scale = p.n_iter / n
    return {"iterations_timed": n, "scaled_to": p.n_iter,
            "total_s": round(sum(ph.values()) * scale, 1),
            **{f"{k}_s": round(v * scale, 1) for k, v in ph.items()}}


def learned_vs_mg(topo, synth, args):
    """The learned preconditioner at the scale of its workload: pairs (r_k, u* - u_k)
    of multigrid-PCG iterates k = 0..19 on random 48x24x24 cantilevers (random
    clamped face, load node and direction, passive boxes, volfrac U[0.15, 0.4],
    rmin U[1.5, 3.0]) at SIMP iterations 1, 5, 10, 20 and 40 of their own
    trajectories; the network trained on the GPU (cosine loss, Adam); then, on
    96x48x48 problems from held-out seeds at the same SIMP iterations, solves to
    1e-8 from zero with plain FP64 MG-PCG, the trained network in flexible CG
    (multigrid restart safeguard), the same network untrained, and Jacobi-PCG,
    plus the held-out loss of the trained and the untrained network."""
    import numpy as np
    import torch
    from synth import networks

    prec = topo.PREC_BF16 if args.learned_precision == "bf16" else topo.PREC_FP32
    t0 = time.perf_counter()
    snaps = [1, 5, 10, 20, 40]
    pair_its = list(range(20))

    def pairs_of(seeds, nelx, its, degree_opts):
        """(rho, r, e, fixed) device tensors, pairs in seed, snapshot, iteration order."""
        probs = []
        for sd in seeds:
            p = synth.random_problem(sd, nelx)
            p.volfrac = float(np.random.default_rng(1000 + sd).uniform(0.15, 0.4))
            probs.append(p)
        V, n = probs[0].nnodes, len(its)
        total = len(probs) * len(snaps) * n
        bufs = (torch.empty(total * V, dtype=torch.float32, device="cuda"),
                torch.empty(total * 3 * V, dtype=torch.float32, device="cuda"),
                torch.empty(total * 3 * V, dtype=torch.float32, device="cuda"),
                torch.empty(total * V, dtype=torch.uint8, device="cuda"))
        k = 0
        for p in probs:
            with topo.Context(p, topo.default_opts(**degree_opts)) as ctx:
                x = torch.from_numpy(p.initial_design()).to("cuda")
                done = 0
                for it in snaps:
                    ctx.iterate(x, it - done, raise_on_nonconv=False)
                    done = it
                    xp = torch.empty(p.nel, dtype=torch.float64, device="cuda")
                    ctx.get_state(xphys=xp)
                    ctx.make_pairs(xp, its, bufs[0][k * V:(k + n) * V], bufs[1][3 * k * V:3 * (k + n) * V],
                                   bufs[2][3 * k * V:3 * (k + n) * V], bufs[3][k * V:(k + n) * V])
                    k += n
        return bufs, total

    # pairs from the degree-2 V-cycle: measured, its iterates train the network
    # to a lower loss than those of the default degrees
    train, n_pairs = pairs_of(range(args.learned_seeds), 48, pair_its, dict(cheb_degree=2, cheb_degree_coarse=2))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    print(f"# learned: {n_pairs} training pairs in {t_data:.1f} s", file=sys.stderr, flush=True)

    w0 = networks.init_weights(seed=0)
    net = topo.Network(precision=prec)
    net.set_weights(w0)
    tr = net.train((49, 25, 25), *train,
                   topo.default_train_opts(epochs=args.learned_epochs, batch=8, lr=1e-3, seed=1, loss=topo.LOSS_COS))
    print(f"# learned: trained {tr['steps']} steps in {tr['ms'] * 1e-3:.1f} s, loss {tr['loss_first']:.3f} -> "
          f"{tr['loss_last']:.3f}", file=sys.stderr, flush=True)
    del train
    torch.cuda.empty_cache()
    untrained = topo.Network(precision=prec)
    untrained.set_weights(w0)

    # held-out loss on pairs of the evaluation problems (96x48x48)
    eval_seeds = list(range(10000, 10000 + args.learned_eval_seeds))
    held, n_held = pairs_of(eval_seeds, 96, [0, 2, 5, 10], dict(cheb_degree=2, cheb_degree_coarse=2))
    nodes96 = (97, 49, 49)
    held_loss = {}
    for name, nw in (("trained", net), ("untrained", untrained)):
        vals = [nw.loss_grad(nodes96, *held, list(range(b, min(n_held, b + 8))), None, loss=topo.LOSS_COS)
                * (min(n_held, b + 8) - b) for b in range(0, n_held, 8)]
        held_loss[name] = round(float(sum(vals) / n_held), 4)
    del held
    torch.cuda.empty_cache()
    print(f"# learned: held-out loss trained {held_loss['trained']}, untrained {held_loss['untrained']}",
          file=sys.stderr, flush=True)

    results = []
    for sd in eval_seeds:
        p = synth.random_problem(sd, 96)
        p.volfrac = float(np.random.default_rng(1000 + sd).uniform(0.15, 0.4))
        with topo.Context(p, topo.default_opts()) as ctx:
            x = torch.from_numpy(p.initial_design()).to("cuda")
            done = 0
            for it in snaps:
                ctx.iterate(x, it - done, raise_on_nonconv=False)
                done = it
                xp = torch.empty(p.nel, dtype=torch.float64, device="cuda")
                ctx.get_state(xphys=xp)
                row = {"seed": sd, "simp_iter": it}
                for name, pc, nn_ in (("mg_fp64", topo.PRECOND_MG, None),
                                      ("learned", topo.PRECOND_LEARNED, net),
                                      ("untrained", topo.PRECOND_LEARNED, untrained),
                                      ("jacobi", topo.PRECOND_JACOBI, None)):
                    o = topo.default_opts(precond=pc, rtol=1e-8, max_iters=5000, nn_max_iters=500)
                    with topo.Context(p, o) as c2:
                        if nn_ is not None:
                            c2.set_nn(nn_)
                        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
                        c2.solve(xp, u, raise_on_nonconv=False)  # captures the CG graphs
                        st = c2.solve(xp, u.zero_(), raise_on_nonconv=False)
                        rec = {"iters": st["iters"], "ms": round(st["ms"], 3), "relres": st["relres"]}
                        if pc == topo.PRECOND_LEARNED:
                            rec.update(learned_iters=st["learned_iters"], fallbacks=st["fallbacks"])
                        row[name] = rec
                results.append(row)
    summary = {k: round(float(np.mean([r[k]["ms"] for r in results])), 3)
               for k in ("mg_fp64", "learned", "untrained", "jacobi")}
    summary["learned_beats_mg"] = sum(1 for r in results if r["learned"]["ms"] < r["mg_fp64"]["ms"])
    summary["solves"] = len(results)
    print(f"# learned: evaluation done ({time.perf_counter() - t0:.1f} s in total), mean ms {summary}",
          file=sys.stderr, flush=True)
    return {
        "train_workload": f"{args.learned_seeds} random cantilevers 48x24x24 (91,875 DOF), pairs at CG "
                          f"iterations 0-19 of SIMP iterations {snaps} (V-cycle of degree 2)",
        "pairs": n_pairs, "pair_gen_s": round(t_data, 2), "epochs": args.learned_epochs, "batch": 8,
        "loss": "cosine", "loss_first_epoch": round(tr["loss_first"], 4), "loss_last_epoch": round(tr["loss_last"], 4),
        "train_s": round(tr["ms"] * 1e-3, 2),
        "train_samples_per_s": round(tr["steps"] * 8 / (tr["ms"] * 1e-3), 1),
        "network_precision": args.learned_precision,
        "held_out_loss": held_loss, "held_out_pairs": n_held,
        "eval_workload": f"random cantilevers 96x48x48 (698,691 DOF), held-out seeds {eval_seeds}, SIMP "
                         f"iterations {snaps}, solve from zero to 1e-8",
        "mean_ms": summary,
        "results": results,
    }


def nn_timing(topo):
    """Times the network alone: forward at 97x49x49 nodes (the 96x48x48
    evaluation grid) and a training step's loss and gradient at 49x25x25 nodes
    (batch 8), BF16 and FP32, with hipEvents around 5 calls each."""
    import numpy as np
    import torch
    from synth import networks

    blob = networks.init_weights(seed=0)
    out = {}
    for prec, name in ((topo.PREC_BF16, "bf16"), (topo.PREC_FP32, "fp32")):
        net = topo.Network(precision=prec)
        net.set_weights(blob)
        nodes = (97, 49, 49)
        V = int(np.prod(nodes))
        g = torch.Generator(device="cuda").manual_seed(0)
        x = torch.randn(4 * V, dtype=torch.float32, device="cuda", generator=g)
        y = torch.empty(3 * V, dtype=torch.float32, device="cuda")
        for _ in range(2):
            net.forward(nodes, 1, x, y)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            net.forward(nodes, 1, x, y)
        b.record()
        torch.cuda.synchronize()
        out[f"{name}_forward_97x49x49_ms"] = round(a.elapsed_time(b) / 5, 3)
        nodes, n = (49, 25, 25), 8
        V = int(np.prod(nodes))
        rho = torch.rand(n * V, device="cuda", generator=g)
        r = torch.randn(n * 3 * V, device="cuda", generator=g)
        e = torch.randn(n * 3 * V, device="cuda", generator=g)
        fx = torch.zeros(n * V, dtype=torch.uint8, device="cuda")
        grad = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
        for _ in range(2):
            net.loss_grad(nodes, rho, r, e, fx, list(range(n)), grad, loss=topo.LOSS_COS)
        t0 = time.perf_counter()
        for _ in range(5):
            net.loss_grad(nodes, rho, r, e, fx, list(range(n)), grad, loss=topo.LOSS_COS)
        torch.cuda.synchronize()
        out[f"{name}_loss_grad_49x25x25_b8_ms"] = round((time.perf_counter() - t0) / 5 * 1e3, 3)
    return out


def lockstep_fp64_error(topo, p, opts, mixed_stats, mixed_ctx):
    """The same SIMP iterations with the FP64 preconditioner from the same initial
    design: largest relative compliance difference over the iterations and the
    relative displacement difference after the last one."""
    import numpy as np
    import torch

    from paper_2504_05604_amd._lib import Opts_C
    opts64 = Opts_C.from_buffer_copy(opts)
    opts64.precision = topo.PREC_FP64
    opts64.mfma_smoothing = 0
    n = len(mixed_stats)
    with topo.Context(p, opts64) as ctx64:
        x64 = torch.from_numpy(p.initial_design()).to("cuda")
        st64 = ctx64.iterate(x64, n, raise_on_nonconv=False)
        u64 = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx64.get_state(u=u64)
    u32 = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
    mixed_ctx.get_state(u=u32)
    c_err = max(abs(a["c"] - b["c"]) / abs(b["c"]) for a, b in zip(mixed_stats, st64))
    u_err = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
    print(f"# FP64 lockstep: max rel compliance difference {c_err:.2e}, rel displacement difference {u_err:.2e}",
          file=sys.stderr, flush=True)
    return {"iterations": n, "compliance_max_rel_diff": float(c_err), "displacement_rel_diff": u_err,
            "fp64_pcg_iters_mean": round(float(np.mean([s["pcg_iters"] for s in st64])), 2)}


def precision_variants(topo, p, opts, args):
    """The mixed-precision configuration's preconditioner variants on the same
    160x80x80 workload: FP64 V-cycle (the reference), FP32 on the vector units
    (the headline mode), FP32 and BF16 operands on the matrix cores.  Each runs
    1 + variant_steps SIMP iterations from the initial design (the first
    untimed); compliance and displacement are compared with the FP64 run."""
    import numpy as np
    import torch

    from paper_2504_05604_amd._lib import Opts_C
    n = args.variant_steps
    modes = (("fp64", topo.PREC_FP64, 0), ("fp32", topo.PREC_FP32, 0), ("fp32_matrix_cores", topo.PREC_FP32, 1),
             ("bf16_matrix_cores", topo.PREC_BF16, 0))
    runs = {}
    for name, prec, mfma in modes:
        o = Opts_C.from_buffer_copy(opts)
        o.precision = prec
        o.mfma_smoothing = mfma
        with topo.Context(p, o) as ctx:
            x = torch.from_numpy(p.initial_design()).to("cuda")
            st = ctx.iterate(x, 1, raise_on_nonconv=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st += ctx.iterate(x, n, raise_on_nonconv=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            u = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
            ctx.get_state(u=u)
        runs[name] = (st, u, 1e3 * dt / n)
    st64, u64, _ = runs["fp64"]
    out = {"workload": "cantilever-160x80x80, the headline options with each preconditioner precision",
           "timed_iterations": n, "untimed_first": 1}
    for name, (st, u, ms) in runs.items():
        out[name] = {
            "ms_per_simp_iteration": round(ms, 3),
            "pcg_iters_mean": round(float(np.mean([s["pcg_iters"] for s in st])), 2),
            "compliance_max_rel_diff_vs_fp64": float(max(abs(a["c"] - b["c"]) / abs(b["c"]) for a, b in zip(st, st64))),
            "displacement_rel_diff_vs_fp64": float(torch.linalg.vector_norm(u - u64) / torch.linalg.vector_norm(u64)),
        }
        print(f"# variant {name}: {ms:.2f} ms per SIMP iteration, "
              f"{out[name]['pcg_iters_mean']} CG iterations", file=sys.stderr, flush=True)
    return out


def batched(topo, synth, args):
    """64 independent random problems (grids 24x12x12 .. 96x48x48, seeds 0-63) with the
    single-precision multigrid preconditioner and autotuned K.u launch shapes:
    aggregate time of one SIMP iteration of the whole batch, driven concurrently
    (one stream per problem, 8 host threads) and one problem after another."""
    import numpy as np
    import torch

    ps = synth.batch_problems(args.batch_size)
    # per-level smoother degrees (finest first; deeper levels take the coarse
    # degree 4): measured on this batch, 143 against 149 ms per batch iteration
    opts = topo.default_opts(precision=topo.PREC_FP32, autotune=1, cheb_degree_level=[1, 2, 4])
    out = {"workload": f"{len(ps)} random cantilevers, seeds 0-{len(ps) - 1}, grids nelx=8*U{{3..12}} x nelx/2 x nelx/2",
           "precond": "mg, fp32 preconditioner, Chebyshev degrees 1, 2, 4 from the finest level down", "autotune": True}
    for label, threads in (("concurrent", 8), ("sequential", 1)):
        t0 = time.perf_counter()
        b = topo.Batch(ps, opts, n_threads=threads)
        out.setdefault("total_dof", int(sum(b.ndof)))
        out.setdefault("setup_s", round(time.perf_counter() - t0, 2))
        print(f"# batched {label}: set up {len(ps)} problems", file=sys.stderr, flush=True)
        xs = [torch.from_numpy(p.initial_design()).to("cuda") for p in ps]
        b.iterate(xs, args.batch_warmup, raise_on_nonconv=False)
        torch.cuda.synchronize()
        print(f"# batched {label}: warm-up done", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        st = b.iterate(xs, args.batch_steps, raise_on_nonconv=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"# batched {label}: timed iterations done", file=sys.stderr, flush=True)
        b.close()
        print(f"# batched {label}: closed", file=sys.stderr, flush=True)
        iters = sum(s["pcg_iters"] for row in st for s in row)
        dof_iters = sum(b.ndof[i] * s["pcg_iters"] for i, row in enumerate(st) for s in row)
        out[label] = {"ms_per_batch_iteration": round(1e3 * dt / args.batch_steps, 2),
                      "pcg_iters_mean": round(iters / (len(ps) * args.batch_steps), 2),
                      "dof_pcg_iters_per_s": round(dof_iters / dt, 1)}
    out["speedup_concurrent_vs_sequential"] = round(
        out["sequential"]["ms_per_batch_iteration"] / out["concurrent"]["ms_per_batch_iteration"], 2)
    print(f"# batched: {out['concurrent']['ms_per_batch_iteration']} ms per batch iteration concurrent, "
          f"{out['sequential']['ms_per_batch_iteration']} sequential", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=28)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precond", choices=["mg", "jacobi"], default="mg")
    ap.add_argument("--cheb-degree", type=int, default=1, help="Chebyshev degree on the finest level")
    ap.add_argument("--cheb-degree-coarse", type=int, default=4, help="Chebyshev degree below the finest level (0: the same)")
    ap.add_argument("--cheb-degree-levels", default="1,2,4,6",
                    help="per-level Chebyshev degrees, finest first, replacing the two above where given "
                         "(measured on the 5-level 160x80x80 hierarchy; '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nn-timing", action="store_true",
                    help="time the network's forward and loss gradient alone and exit")
    ap.add_argument("--record-oracle-iteration", action="store_true",
                    help="time one complete oracle SIMP iteration at 160x80x80 on the host (minutes), "
                         "write its record under profiles/ and exit (no GPU work)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--ku-reps", type=int, default=100)
    ap.add_argument("--coarse-dof", type=int, default=1500, help="coarsest multigrid level size cap")
    ap.add_argument("--check-every", type=int, default=3)
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp32",
                    help="precision of the multigrid preconditioner (CG stays FP64)")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="skip the lockstep FP64 run that measures the mixed-precision error")
    ap.add_argument("--mfma", action="store_true",
                    help="FP32 preconditioner: smoothing operator passes on the matrix cores")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed run, copy a buffer of this many MiB 5 times (a plain copy "
                         "kernel of known traffic for calibrating hardware byte counters)")
    ap.add_argument("--tail-nodes", type=int, default=0,
                    help="levels with at most this many nodes run as one single-workgroup launch (0 = off)")
    ap.add_argument("--warm", type=int, default=3, choices=[0, 1, 2, 3],
                    help="initial guess of each solve: 0 zero, 1 last solution, 2 extrapolated, 3 projected")
    ap.add_argument("--autotune", action="store_true", help="time every K.u launch shape at set-up")
    ap.add_argument("--ku-kernel", choices=["auto", "node", "element"], default="auto",
                    help="K.u kernel: node columns or element columns in the sum/difference basis")
    ap.add_argument("--ku-shape", type=int, default=-1, help="one K.u launch shape for every level (-1: by grid size)")
    ap.add_argument("--cheb-upper", type=float, default=0.7,
                    help="top of the smoothing interval as a fraction of the element bound (1: the bound)")
    ap.add_argument("--coarse-refresh", type=int, default=2,
                    help="recompute the coarsest level's dense inverse every this many SIMP iterations "
                         "(in between the previous one, still SPD, preconditions)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-multigrid leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems leg")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's 32x16x16 workload")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the preconditioner-precision variants of the 160x80x80 workload")
    ap.add_argument("--variant-steps", type=int, default=3)
    ap.add_argument("--batch-size", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--learned-seeds", type=int, default=200,
                    help="random 48x24x24 training problems (100 pairs each)")
    ap.add_argument("--learned-epochs", type=int, default=3)
    ap.add_argument("--learned-eval-seeds", type=int, default=2, help="held-out 96x48x48 problems")
    ap.add_argument("--learned-precision", choices=["bf16", "fp32"], default="bf16")
    args = ap.parse_args()
    if args.nn_timing:
        import paper_2504_05604_amd as topo
        print(json.dumps({"nn_timing": nn_timing(topo)}))
        return
    if args.record_oracle_iteration:
        import synth
        record_oracle_iteration(synth.config_large())
        return
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus above 1 is not supported "
              "(the multi-GPU decomposition is described in DESIGN.md, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2504_05604_amd as topo
    import synth

    p = synth.config_large()
    level_degs = [int(v) for v in args.cheb_degree_levels.split(",") if v.strip()]
    opts = topo.default_opts(rtol=1e-8, max_iters=2000, cheb_degree=args.cheb_degree, warm_start=args.warm,
                             cheb_degree_coarse=args.cheb_degree_coarse, cheb_degree_level=level_degs,
                             mg_max_coarse_dof=args.coarse_dof, check_every=args.check_every,
                             use_graphs=0 if args.no_graphs else 1, coarse_tail_nodes=args.tail_nodes,
                             precision={"fp64": topo.PREC_FP64, "fp32": topo.PREC_FP32,
                                        "bf16": topo.PREC_BF16}[args.precision],
                             mfma_smoothing=1 if args.mfma else 0, autotune=1 if args.autotune else 0,
                             ku_kernel={"auto": topo.KU_AUTO, "node": topo.KU_NODE,
                                        "element": topo.KU_ELEMENT}[args.ku_kernel],
                             ku_shape=args.ku_shape, coarse_refresh=args.coarse_refresh,
                             cheb_upper=args.cheb_upper,
                             precond=topo.PRECOND_MG if args.precond == "mg" else topo.PRECOND_JACOBI)
    ctx = topo.Context(p, opts)
    x = torch.from_numpy(p.initial_design()).to("cuda")
    print(f"# setup done: {p.nel} elements, {p.ndof} dof, {ctx.mg_levels} MG levels", file=sys.stderr, flush=True)
    warm_stats = ctx.iterate(x, args.warmup, raise_on_nonconv=False) if args.warmup else []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = ctx.iterate(x, args.steps, raise_on_nonconv=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    print(f"# timed {args.steps} SIMP iterations: {ms_per_step:.2f} ms each", file=sys.stderr, flush=True)
    fp64_reference = None
    if args.precision != "fp64" and not args.no_fp64_reference:
        fp64_reference = lockstep_fp64_error(topo, p, opts, warm_stats + stats, ctx)

    pcg = np.array([s["pcg_iters"] for s in stats], dtype=float)
    solve_ms = np.array([s["ms_solve"] for s in stats])
    deg = args.cheb_degree
    # fine-grid K.u applications per CG iteration: the product itself plus 2 deg_l
    # on each smoothed level l of the V-cycle, level l costing 8^-l of the finest
    degc = args.cheb_degree_coarse or deg
    ku_per_cg = 1.0
    if args.precond == "mg":
        for lvl in range(ctx.mg_levels - 1):
            d = level_degs[lvl] if lvl < len(level_degs) and level_degs[lvl] > 0 else (deg if lvl == 0 else degc)
            ku_per_cg += 2.0 * d / 8.0 ** lvl
    ku_equiv = float(pcg.mean() * ku_per_cg + 1.0)

    ku_ms = ctx.time_operator(args.ku_reps)
    kernel = {"node": "ku_march_kernel (node columns", "element": "ku_hada_kernel (element columns",
              "auto": "ku_hada_kernel (element columns"}[args.ku_kernel]
    achieved = ku_algorithmic_bytes(p) / (ku_ms * 1e-3) / 1e9
    roofline = {
        "kernel": kernel + ", finest-level K.u, y = K u, FP64)",
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": ku_traffic_bytes() if args.ku_kernel != "node" and args.ku_shape < 0 else None,
        "algorithmic_bytes": ku_algorithmic_bytes(p), "ms_per_launch": round(ku_ms, 5),
    }

    out = {
        "metric": METRIC,
        "value": round(ms_per_step, 3),
        "unit": "ms/SIMP iteration",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64/f32", "bf16": "f64/bf16"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": "cantilever-160x80x80 (3,168,963 DOF), volfrac 0.2, rmin 3.0, density filter",
            "nel": p.nel, "ndof": p.ndof, "precond": args.precond, "mg_levels": ctx.mg_levels,
            "cheb_degree": deg, "cheb_degree_coarse": args.cheb_degree_coarse or deg,
            "cheb_degree_level": level_degs, "rtol": 1e-8, "warm_start": ["zero", "last", "extrapolated", "projected"][args.warm],
            "coarse_dof_cap": args.coarse_dof,
            "check_every": args.check_every, "graphs": not args.no_graphs,
            "coarse_tail_nodes": args.tail_nodes, "autotune": bool(args.autotune),
            "cheb_upper": args.cheb_upper,
            "ku_kernel": args.ku_kernel, "ku_shape": args.ku_shape, "coarse_refresh": args.coarse_refresh,
            "preconditioner_precision": args.precision,
            "error_vs_fp64": fp64_reference,
            "matrix_core_smoothing": bool(args.mfma or args.precision == "bf16"),
            "pcg_iters_mean": round(float(pcg.mean()), 2), "pcg_iters_max": int(pcg.max()),
            "solves_converged": int(sum(1 for s in stats if s["converged"])),
            "solve_ms_mean": round(float(solve_ms.mean()), 3),
            "dof_pcg_iters_per_s": round(float(p.ndof * pcg.sum() / (solve_ms.sum() * 1e-3)), 1),
            "phase_ms_mean": {k: round(float(np.mean([s[k] for s in stats])), 3)
                              for k in ("ms_filter", "ms_solve", "ms_sens", "ms_oc")},
            "compliance_last": stats[-1]["c"],
            "precision_variants": None,
            "learned_vs_mg": None,
            "batched": None,
            "paper_benchmark": None,
        },
        "roofline": roofline,
    }
    ctx.close()
    if not args.no_variants:
        out["config"]["precision_variants"] = precision_variants(topo, p, opts, args)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_learned:
        out["config"]["learned_vs_mg"] = learned_vs_mg(topo, synth, args)
    if not args.no_batch:
        out["config"]["batched"] = batched(topo, synth, args)
    if not args.no_paper:
        out["config"]["paper_benchmark"] = paper_benchmark(topo, synth, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, ku_equiv, args.cpu_budget)
        if not args.no_paper:
            out["cpu_baseline"]["paper_benchmark_oracle"] = paper_benchmark_oracle(args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
