"""GPU parity of the matrix-free stiffness operator for every launch shape of both
K.u kernels (node columns, and element columns in the sum/difference basis),
against the CPU FP64 oracle: ragged tiles and slabs, grids smaller than one
tile, single-element-thick grids, and the full 160x80x80 grid."""

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.ke import element_stiffness

torch = pytest.importorskip("torch")
import paper_2504_05604_amd as topo  # noqa: E402

pytestmark = pytest.mark.gpu
KE = element_stiffness(0.3)

# launch shapes: 0..3 node-column kernel, 6..14 element-column kernel
SHAPES = [0, 1, 2, 3, 6, 7, 8, 9, 10, 11, 12, 13, 14]
# ragged in every tile and slab size of both kernels, smaller than one tile, one element thick
GRIDS = [(37, 21, 19), (5, 3, 4), (1, 1, 1), (40, 1, 3), (2, 17, 1)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problem(dims, seed):
    p = synth.cantilever(*dims, volfrac=0.3, rmin=1.5, n_iter=5)
    rng = np.random.default_rng(seed)
    extra = rng.choice(p.ndof, min(5, p.ndof // 4), replace=False)
    p.fixed_dofs = np.unique(np.concatenate([p.fixed_dofs, extra])).astype(np.int64)
    return p


def apply_K(p, x, u, **opts):
    # the operator alone: no multigrid hierarchy needed (also for one-element grids)
    with topo.Context(p, topo.default_opts(precond=topo.PRECOND_JACOBI, **opts)) as ctx:
        y = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
        ctx.apply_K(dev(x), dev(u), y)
        return host(y)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dims", GRIDS)
def test_every_launch_shape_matches_oracle(dims, shape):
    p = problem(dims, 1)
    x = synth.random_density(2, p.nel, 0.0, 1.0)
    u = synth.random_vector(3, p.ndof)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    ref = fem.apply_K_reduced(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), u, p.fixed_dofs)
    got = apply_K(p, x, u, ku_shape=shape)
    print(dims, shape, "max rel err", np.abs(got - ref).max() / np.abs(ref).max())
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_every_launch_shape_solves(shape):
    """All fused epilogues (CG product with its dot product, every Chebyshev
    step, residuals) of one launch shape on every level: the solve reaches the
    tolerance and its true residual, computed by the oracle, agrees."""
    p = problem((37, 21, 19), 4)
    p.f = synth.random_vector(5, p.ndof)
    x = synth.random_density(6, p.nel, 0.05, 1.0)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    f = p.f.copy()
    f[p.fixed_dofs] = 0.0
    with topo.Context(p, topo.default_opts(rtol=1e-10, max_iters=2000, ku_shape=shape,
                                           coarse_tail_nodes=0)) as ctx:
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        st = ctx.solve(dev(x), u)
        got = host(u)
    assert st["converged"]
    res = f - fem.apply_K_reduced(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), got, p.fixed_dofs)
    assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(f)


def test_kernels_agree_in_iterations():
    """Same solve with the two kernels: the same iteration count (give or take the
    one that rounding can move across the tolerance) and solutions within the
    solver tolerance (the products differ only by rounding)."""
    p = problem((37, 21, 19), 7)
    p.f = synth.random_vector(8, p.ndof)
    x = synth.random_density(9, p.nel, 0.05, 1.0)
    out = {}
    for k in (topo.KU_NODE, topo.KU_ELEMENT):
        with topo.Context(p, topo.default_opts(rtol=1e-10, ku_kernel=k)) as ctx:
            u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
            st = ctx.solve(dev(x), u)
            out[k] = (host(u), st["iters"])
    assert abs(out[topo.KU_NODE][1] - out[topo.KU_ELEMENT][1]) <= 1
    un, ue = out[topo.KU_NODE][0], out[topo.KU_ELEMENT][0]
    assert np.linalg.norm(un - ue) <= 1e-8 * np.linalg.norm(un)


@pytest.mark.parametrize("kernel", [topo.KU_ELEMENT, topo.KU_NODE])
def test_full_size_operator_matches_oracle(kernel):
    """160x80x80 (3,168,963 dofs), the launch shapes the solver uses there, every
    output compared (the oracle's elementwise product takes well under a second)."""
    p = synth.config_large()
    x = synth.random_density(11, p.nel, 0.0, 1.0)
    u = synth.random_vector(12, p.ndof)
    E = fem.simp_modulus(x, p.E0, p.Emin, p.penal)
    ref = fem.apply_K_reduced(E, KE, fem.element_dofs(p.nelx, p.nely, p.nelz), u, p.fixed_dofs)
    got = apply_K(p, x, u, ku_kernel=kernel)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("kernel", kernel, "max rel err", err)
    assert err <= 1e-13
