"""GPU parity of the convolutional preconditioner network and of the learned
preconditioner inside flexible CG, against the FP64 oracle (oracle.nn,
oracle.fpcg) on the same seeded inputs.

Tolerances: the network runs in FP32 with FP32 accumulation.  Each output is a
sum of at most 27 * 128 = 3456 products per layer over 11 layers; with
unit-scale activations the rounding error of such sums grows like
sqrt(K) * 2^-24 per layer, about 3e-5 of the output scale over the whole
network, so forward outputs are compared at 2e-4 of their maximum magnitude.
Parameter gradients sum up to batch * V ~ 1e5 products (in split slices whose
partials are added in a fixed order); they are compared per layer in the
relative 2-norm at 1e-3.
"""

import numpy as np
import pytest

import synth
from synth import networks
from oracle import fem, fpcg, mg, nn
from oracle.ke import element_stiffness

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu
KE = element_stiffness(0.3)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_params(blob, ch):
    return nn.unpack(blob.astype(np.float64), ch)


@pytest.mark.parametrize("ch,nodes,batch", [
    ((16, 32, 64), (9, 7, 6), 1),
    ((16, 32, 64), (21, 11, 13), 2),
    ((3, 5, 7), (6, 9, 5), 3),
])
def test_forward_matches_oracle(ch, nodes, batch):
    blob = networks.init_weights(ch, seed=1)
    x = networks.random_activations(2, 4, batch, nodes)
    net = topo.Network(ch)
    net.set_weights(blob)
    V = int(np.prod(nodes))
    out = torch.empty(3 * batch * V, dtype=torch.float32, device="cuda")
    net.forward(nodes, batch, dev(x.reshape(-1)), out)
    got = host(out).reshape(3, batch, nodes[2], nodes[1], nodes[0])
    P = oracle_params(blob, ch)
    for b in range(batch):
        ref = nn.forward(P, x[:, b].astype(np.float64))
        assert np.abs(got[:, b] - ref).max() <= 2e-4 * np.abs(ref).max(), b


@pytest.mark.parametrize("ch,nodes,batch", [
    ((16, 32, 64), (9, 7, 6), 1),
    ((16, 32, 64), (21, 11, 13), 2),
    ((3, 5, 7), (6, 9, 5), 3),
])
def test_bf16_forward_matches_oracle(ch, nodes, batch):
    """BF16 operands (8-bit mantissa, relative rounding 2^-9) with FP32
    accumulation: each layer's output carries a relative error of about
    2^-9 sqrt(#layers); compared at 3e-2 of the output scale."""
    blob = networks.init_weights(ch, seed=1)
    x = networks.random_activations(2, 4, batch, nodes)
    net = topo.Network(ch, precision=topo.PREC_BF16)
    net.set_weights(blob)
    V = int(np.prod(nodes))
    out = torch.empty(3 * batch * V, dtype=torch.float32, device="cuda")
    net.forward(nodes, batch, dev(x.reshape(-1)), out)
    got = host(out).reshape(3, batch, nodes[2], nodes[1], nodes[0])
    P = oracle_params(blob, ch)
    for b in range(batch):
        ref = nn.forward(P, x[:, b].astype(np.float64))
        err = np.abs(got[:, b] - ref).max() / np.abs(ref).max()
        rel2 = np.linalg.norm(got[:, b] - ref) / np.linalg.norm(ref)
        print("bf16 forward max err", err, "rel2", rel2)
        assert err <= 3e-2 and rel2 <= 1e-2, b


def node_fixed_bits(fixed_mask_dof):
    m = fixed_mask_dof.reshape(-1, 3)
    return (m[:, 0] * 1 + m[:, 1] * 2 + m[:, 2] * 4).astype(np.uint8)


def random_samples(seed, n, nodes):
    rng = np.random.default_rng(seed)
    V = int(np.prod(nodes))
    rho = rng.uniform(0, 1, (n, V)).astype(np.float32)
    r = rng.standard_normal((n, 3 * V)).astype(np.float32)
    e = rng.standard_normal((n, 3 * V)).astype(np.float32)
    fixed = np.zeros((n, 3 * V), bool)
    for i in range(n):
        fixed[i, rng.choice(3 * V, 3 * V // 10, replace=False)] = True
    r[fixed] = 0.0
    return rho, r, e, fixed


@pytest.mark.parametrize("mode", ["rel", "cos"])
@pytest.mark.parametrize("nodes,batch", [((9, 7, 6), 1), ((13, 7, 9), 3)])
def test_loss_gradient_matches_oracle(nodes, batch, mode):
    ch = (16, 32, 64)
    blob = networks.init_weights(ch, seed=3)
    n = batch + 1
    rho, r, e, fixed = random_samples(4, n, nodes)
    index = np.arange(1, n)[:batch]
    net = topo.Network(ch)
    net.set_weights(blob)
    grad = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    bits = np.stack([node_fixed_bits(f) for f in fixed])
    loss = net.loss_grad(nodes, dev(rho.reshape(-1)), dev(r.reshape(-1)), dev(e.reshape(-1)),
                         dev(bits.reshape(-1), torch.uint8), index, grad,
                         loss=topo.LOSS_REL if mode == "rel" else topo.LOSS_COS)
    g = host(grad)
    P = oracle_params(blob, ch)
    shape = (nodes[2], nodes[1], nodes[0])
    ref_loss, ref_g = 0.0, None
    for i in index:
        l, gi = nn.loss_and_grad(P, rho[i].astype(np.float64).reshape(shape), r[i].astype(np.float64),
                                 e[i].astype(np.float64), fixed[i], mode)
        vec = nn.pack(gi, ch)
        ref_loss += l / batch
        ref_g = vec / batch if ref_g is None else ref_g + vec / batch
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    off = 0
    for name, wshape, nb in networks.layer_shapes(ch):
        k = int(np.prod(wshape)) + nb
        a, b = g[off:off + k], ref_g[off:off + k]
        print("fp32 grad", mode, name, np.linalg.norm(a - b) / np.linalg.norm(b))
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b), name
        off += k


@pytest.mark.parametrize("mode", ["rel", "cos"])
def test_bf16_loss_gradient_matches_oracle(mode):
    """BF16 products in every backward GEMM.  The parameter gradients of a
    random-initialised network are sums with heavy cancellation, so their
    relative error is the operand rounding (2^-9, 2^15 times FP32's) amplified
    by the cancellation; the FP32 kernels show about 1e-6 per layer on this case,
    so BF16 is held to 0.15 per layer in the relative 2-norm, and to a cosine of
    at least 0.995 between the whole gradient vectors."""
    ch = (16, 32, 64)
    nodes, batch = (13, 7, 9), 3
    blob = networks.init_weights(ch, seed=3)
    n = batch + 1
    rho, r, e, fixed = random_samples(4, n, nodes)
    index = np.arange(1, n)[:batch]
    net = topo.Network(ch, precision=topo.PREC_BF16)
    net.set_weights(blob)
    grad = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    bits = np.stack([node_fixed_bits(f) for f in fixed])
    loss = net.loss_grad(nodes, dev(rho.reshape(-1)), dev(r.reshape(-1)), dev(e.reshape(-1)),
                         dev(bits.reshape(-1), torch.uint8), index, grad,
                         loss=topo.LOSS_REL if mode == "rel" else topo.LOSS_COS)
    g = host(grad)
    P = oracle_params(blob, ch)
    shape = (nodes[2], nodes[1], nodes[0])
    ref_loss, ref_g = 0.0, 0.0
    for i in index:
        l, gi = nn.loss_and_grad(P, rho[i].astype(np.float64).reshape(shape), r[i].astype(np.float64),
                                 e[i].astype(np.float64), fixed[i], mode)
        ref_loss += l / batch
        ref_g = ref_g + nn.pack(gi, ch) / batch
    assert abs(loss - ref_loss) <= 1e-2 * abs(ref_loss)
    off = 0
    for name, wshape, nb in networks.layer_shapes(ch):
        k = int(np.prod(wshape)) + nb
        a, b = g[off:off + k], ref_g[off:off + k]
        print("bf16 grad", mode, name, np.linalg.norm(a - b) / np.linalg.norm(b))
        assert np.linalg.norm(a - b) <= 0.15 * np.linalg.norm(b), name
        off += k
    cos = float(g @ ref_g) / (np.linalg.norm(g) * np.linalg.norm(ref_g))
    print("bf16 grad cosine", mode, cos)
    assert cos >= 0.995


def test_adam_step_matches_oracle_gradient():
    """One Adam step from zero moments moves every weight by -lr g / (|g| + eps)."""
    ch = (16, 32, 64)
    nodes = (9, 7, 6)
    blob = networks.init_weights(ch, seed=5)
    rho, r, e, fixed = random_samples(6, 2, nodes)
    net = topo.Network(ch)
    net.set_weights(blob)
    bits = np.stack([node_fixed_bits(f) for f in fixed])
    lr = 1e-3
    opts = topo.default_train_opts(epochs=1, batch=2, lr=lr, seed=0)
    st = net.train(nodes, dev(rho.reshape(-1)), dev(r.reshape(-1)), dev(e.reshape(-1)),
                   dev(bits.reshape(-1), torch.uint8), opts)
    assert st["steps"] == 1
    w1 = net.get_weights().astype(np.float64)
    P = oracle_params(blob, ch)
    shape = (nodes[2], nodes[1], nodes[0])
    g = 0.0
    for i in range(2):
        _, gi = nn.loss_and_grad(P, rho[i].astype(np.float64).reshape(shape), r[i].astype(np.float64),
                                 e[i].astype(np.float64), fixed[i])
        g = g + nn.pack(gi, ch) / 2
    step = w1 - blob.astype(np.float64)
    assert np.all(np.abs(step) <= lr * (1 + 1e-5) + 1e-7)
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    ref = -lr * g / (np.abs(g) + 1e-8)
    assert np.abs(step[big] - ref[big]).max() <= 1e-5 * lr + 2e-7


def identity_weights(ch=(16, 32, 64)):
    """A network whose output is exactly its residual input: r = relu(r) - relu(-r)
    carried through enc0a, enc0b, dec0 and the head; every other layer is zero."""
    parts = {}
    for name, w, nb in networks.layer_shapes(ch):
        parts[name] = (np.zeros(w), np.zeros(nb))
    c0 = ch[0]
    for c in range(3):
        parts["enc0a"][0][c, 1 + c, 1, 1, 1] = 1.0
        parts["enc0a"][0][3 + c, 1 + c, 1, 1, 1] = -1.0
    for j in range(6):
        parts["enc0b"][0][j, j, 1, 1, 1] = 1.0
        parts["dec0"][0][j, c0 + j, 1, 1, 1] = 1.0
    for c in range(3):
        parts["head"][0][c, c, 0, 0, 0] = 1.0
        parts["head"][0][c, 3 + c, 0, 0, 0] = -1.0
    return np.concatenate([np.concatenate([parts[n][0].ravel(), parts[n][1].ravel()])
                           for n, _, _ in networks.layer_shapes(ch)]).astype(np.float32)


def small_problem():
    p = synth.config_small()
    x = synth.random_density(7, p.nel, 0.3, 1.0)
    return p, x


def fixed_mask(p):
    fm = np.zeros(p.ndof, bool)
    fm[p.fixed_dofs] = True
    return fm


def test_learned_preconditioner_application_matches_oracle():
    p, x = small_problem()
    ch = (16, 32, 64)
    blob = networks.init_weights(ch, seed=8)
    fm = fixed_mask(p)
    r = synth.random_vector(9, p.ndof)
    r[fm] = 0.0
    opts = topo.default_opts(precond=topo.PRECOND_LEARNED)
    net = topo.Network(ch)
    net.set_weights(blob)
    with topo.Context(p, opts) as ctx:
        ctx.set_nn(net)
        z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(x, torch.float64), dev(r, torch.float64), z)
        got = host(z)
    rho = nn.node_density(x, p.nelx, p.nely, p.nelz)
    ref = nn.apply(oracle_params(blob, ch), rho, r, fm)
    assert np.abs(got - ref).max() <= 2e-4 * np.abs(ref).max()
    assert np.all(got[fm] == 0.0)


def direct_solution(p, x):
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    K = fem.assemble(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), p.ndof)
    return fem.solve(K, p.f, p.fixed_dofs), K


def test_identity_network_gives_plain_cg():
    """z = r makes flexible CG plain CG: same solution as the direct solve, and the
    iteration count of the oracle's flexible CG with the same preconditioner.  The
    network sees r / rms(r) rounded to FP32, so the oracle preconditioner is that
    rounding, rescaled (exact identity takes fewer iterations)."""
    p, x = small_problem()
    blob = identity_weights()
    fm = fixed_mask(p)
    # the oracle network reproduces its input exactly
    rho = nn.node_density(x, p.nelx, p.nely, p.nelz)
    rr = synth.random_vector(10, p.ndof)
    rr[fm] = 0.0
    assert np.abs(nn.apply(oracle_params(blob, (16, 32, 64)), rho, rr, fm) - rr).max() <= 1e-14 * np.abs(rr).max()
    opts = topo.default_opts(precond=topo.PRECOND_LEARNED, rtol=1e-10, max_iters=6000, nn_max_iters=5000)
    net = topo.Network()
    net.set_weights(blob)
    with topo.Context(p, opts) as ctx:
        ctx.set_nn(net)
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        st = ctx.solve(dev(x, torch.float64), u)
        got = host(u)
    us, K = direct_solution(p, x)
    assert st["fallbacks"] == 0 and st["learned_iters"] == st["iters"]
    assert np.abs(got - us).max() <= 1e-8 * np.abs(us).max()
    free = ~fm
    A = K[free][:, free]
    n_all = p.ndof

    def rounded(v):
        s = np.sqrt((v @ v) / n_all)
        return s * (v / s).astype(np.float32).astype(np.float64)

    _, it, _, fb, _ = fpcg.fpcg(A, p.f[free], rounded, lambda v: v, rtol=1e-10, max_iter=6000,
                                nn_max_iter=5000)
    print("GPU iterations", st["iters"], "oracle", it)
    assert fb == 0 and abs(st["iters"] - it) <= max(3, 0.05 * it)


@pytest.mark.parametrize("bad", ["nan", "zero", "negated"])
def test_failing_network_falls_back_to_multigrid(bad):
    p, x = small_problem()
    blob = identity_weights()
    if bad == "nan":
        blob[:] = np.nan
    elif bad == "zero":
        blob[:] = 0.0
    else:
        lay = networks.layer_shapes()
        head_off = sum(int(np.prod(w)) + b for _, w, b in lay[:-1])
        blob[head_off:head_off + 3 * 16] *= -1.0
    opts = topo.default_opts(precond=topo.PRECOND_LEARNED, rtol=1e-10)
    net = topo.Network()
    net.set_weights(blob)
    with topo.Context(p, opts) as ctx:
        ctx.set_nn(net)
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        st = ctx.solve(dev(x, torch.float64), u)
        got = host(u)
    us, _ = direct_solution(p, x)
    assert st["fallbacks"] == 1 and st["learned_iters"] == 0 and st["converged"]
    assert np.abs(got - us).max() <= 1e-8 * np.abs(us).max()


def test_training_pairs_match_oracle_iterates():
    """Pairs (r_k, u* - u_k): u_k is the k-th multigrid-PCG iterate from zero.  The
    oracle runs the same V-cycle (its own implementation) and CG."""
    p = synth.random_problem(3, 16, boxes=1)
    x = synth.random_density(11, p.nel, 0.2, 1.0)
    iters = np.array([0, 1, 2, 5], np.int32)
    # the same hierarchy and smoother as the oracle's V-cycle below
    opts = topo.default_opts(precond=topo.PRECOND_MG, mg_max_coarse_dof=140, cheb_degree=2, cheb_degree_coarse=2)
    V = p.nnodes
    n = iters.size
    rho = torch.empty(n * V, dtype=torch.float32, device="cuda")
    r = torch.empty(n * 3 * V, dtype=torch.float32, device="cuda")
    e = torch.empty(n * 3 * V, dtype=torch.float32, device="cuda")
    fixed = torch.empty(n * V, dtype=torch.uint8, device="cuda")
    with topo.Context(p, opts) as ctx:
        ctx.make_pairs(dev(x, torch.float64), iters, rho, r, e, fixed)
    rho, r, e, fixed = host(rho), host(r).reshape(n, -1), host(e).reshape(n, -1), host(fixed)
    fm = fixed_mask(p)
    assert np.array_equal(fixed.reshape(n, V)[0], node_fixed_bits(fm))
    ref_rho = nn.node_density(x, p.nelx, p.nely, p.nelz).ravel()
    assert np.abs(rho[:V] - ref_rho).max() <= 1e-7
    us, K = direct_solution(p, x)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    vc = mg.VCycle(p, E, KE, degree=2, max_coarse_dof=140)
    Kr = mg.with_identity_rows(K, fm)
    f = p.f.copy()
    f[fm] = 0.0
    for i, k in enumerate(iters):
        uk, _, _ = mg.pcg(Kr, f, M=vc.apply, rtol=0.0, max_iter=int(k))
        rk = f - Kr @ uk
        ek = us - uk
        assert np.abs(e[i] - ek).max() <= 1e-5 * np.abs(ek).max(), k
        assert np.abs(r[i] - rk).max() <= 1e-5 * np.abs(rk).max(), k


def test_training_reduces_loss():
    p = synth.random_problem(4, 16, boxes=0)
    x = synth.random_density(12, p.nel, 0.2, 1.0)
    iters = np.array([0, 1, 2, 3, 4, 6, 8, 10], np.int32)
    V = p.nnodes
    n = iters.size
    rho = torch.empty(n * V, dtype=torch.float32, device="cuda")
    r = torch.empty(n * 3 * V, dtype=torch.float32, device="cuda")
    e = torch.empty(n * 3 * V, dtype=torch.float32, device="cuda")
    fixed = torch.empty(n * V, dtype=torch.uint8, device="cuda")
    with topo.Context(p, topo.default_opts()) as ctx:
        ctx.make_pairs(dev(x, torch.float64), iters, rho, r, e, fixed)
    net = topo.Network()
    net.set_weights(networks.init_weights(seed=13))
    nodes = (p.nelx + 1, p.nely + 1, p.nelz + 1)
    st = net.train(nodes, rho, r, e, fixed, topo.default_train_opts(epochs=40, batch=4, lr=1e-3, seed=1))
    assert st["steps"] == 80
    print("epoch losses", ["%.4f" % v for v in st["epoch_loss"]])
    assert np.all(np.isfinite(st["epoch_loss"]))
    assert st["loss_last"] < st["loss_first"]


def simp_pairs(seeds, nelx, snaps, pair_its):
    """Training pairs (node density, r_k, u* - u_k) from the multigrid-PCG
    iterates k of random cantilevers (volfrac U[0.15, 0.4]) at SIMP iterations
    `snaps` of their own trajectories."""
    parts = []
    for s in seeds:
        p = synth.random_problem(s, nelx)
        p.volfrac = float(np.random.default_rng(1000 + s).uniform(0.15, 0.4))
        V, n = p.nnodes, len(pair_its)
        with topo.Context(p, topo.default_opts(cheb_degree=2, cheb_degree_coarse=2)) as ctx:
            x = dev(p.initial_design(), torch.float64)
            done = 0
            for it in snaps:
                ctx.iterate(x, it - done, raise_on_nonconv=False)
                done = it
                xp = torch.empty(p.nel, dtype=torch.float64, device="cuda")
                ctx.get_state(xphys=xp)
                bufs = (torch.empty(n * V, dtype=torch.float32, device="cuda"),
                        torch.empty(n * 3 * V, dtype=torch.float32, device="cuda"),
                        torch.empty(n * 3 * V, dtype=torch.float32, device="cuda"),
                        torch.empty(n * V, dtype=torch.uint8, device="cuda"))
                ctx.make_pairs(xp, pair_its, *bufs)
                parts.append(bufs)
    return tuple(torch.cat([b[i] for b in parts]) for i in range(4))


def test_trained_network_gains_over_the_untrained_one():
    """What training gains, on held-out problems: a BF16 network trained on pairs
    from 64 random 24x12x12 cantilevers (cosine loss) against the same network at
    its initial weights, on pairs from 3 unseen seeds (>= 10000) -- the held-out
    loss, 1 - cos(net(r), K^-1 r) on the free dofs -- and inside flexible CG on an
    unseen problem, where the safeguard accepts the trained network's directions
    for more iterations."""
    nodes = (25, 13, 13)
    snaps, pair_its = [1, 5, 10], [0, 1, 2, 4, 6, 8]
    train = simp_pairs(range(64), 24, snaps, pair_its)
    held = simp_pairs([10000, 10001, 10003], 24, snaps, pair_its)
    w0 = networks.init_weights(seed=0)
    trained = topo.Network(precision=topo.PREC_BF16)
    trained.set_weights(w0)
    st = trained.train(nodes, *train, topo.default_train_opts(epochs=6, batch=8, lr=1e-3, seed=1,
                                                                loss=topo.LOSS_COS))
    untrained = topo.Network(precision=topo.PREC_BF16)
    untrained.set_weights(w0)
    n_held = held[0].numel() // int(np.prod(nodes))
    idx = np.arange(n_held)
    l_tr = trained.loss_grad(nodes, *held, idx, None, loss=topo.LOSS_COS)
    l_un = untrained.loss_grad(nodes, *held, idx, None, loss=topo.LOSS_COS)
    print(f"training loss {st['loss_first']:.3f} -> {st['loss_last']:.3f}; held-out loss trained {l_tr:.3f}, "
          f"untrained {l_un:.3f}")
    assert l_tr < l_un - 0.1
    # inside flexible CG on an unseen problem at SIMP iteration 5
    p = synth.random_problem(10002, 24)
    with topo.Context(p, topo.default_opts()) as ctx:
        x = dev(p.initial_design(), torch.float64)
        ctx.iterate(x, 5)
        xp = torch.empty(p.nel, dtype=torch.float64, device="cuda")
        ctx.get_state(xphys=xp)
    res = {}
    for name, net in (("trained", trained), ("untrained", untrained)):
        with topo.Context(p, topo.default_opts(precond=topo.PRECOND_LEARNED, rtol=1e-8, max_iters=2000,
                                               nn_max_iters=500)) as ctx:
            ctx.set_nn(net)
            u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
            res[name] = ctx.solve(xp, u)
    print("flexible CG", res)
    assert res["trained"]["converged"] and res["untrained"]["converged"]
    assert res["trained"]["learned_iters"] > res["untrained"]["learned_iters"]
