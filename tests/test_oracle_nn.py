"""Pins of the FP64 oracle of the convolutional preconditioner network: against
torch's CPU convolution routines (an independent library), the adjoint
identity, and central finite differences of the training loss."""

import numpy as np
import pytest

from oracle import nn

torch = pytest.importorskip("torch")
F = torch.nn.functional


def rnd(seed, *shape):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("stride", [1, 2])
@pytest.mark.parametrize("shape", [(5, 4, 6), (6, 6, 3)])
def test_conv_matches_torch(stride, shape):
    x, W, b = rnd(1, 3, *shape), rnd(2, 5, 3, 3, 3, 3), rnd(3, 5)
    ref = F.conv3d(torch.from_numpy(x)[None], torch.from_numpy(W), torch.from_numpy(b),
                   stride=stride, padding=1)[0].numpy()
    np.testing.assert_allclose(nn.conv(x, W, b, stride), ref, atol=1e-12)


@pytest.mark.parametrize("shape", [(5, 4, 6), (6, 6, 3), (7, 3, 2)])
def test_up_matches_torch_transpose(shape):
    coarse = tuple(-(-n // 2) for n in shape)
    x, W, b = rnd(4, 5, *coarse), rnd(5, 5, 3, 3, 3, 3), rnd(6, 3)
    op = tuple(1 if n % 2 == 0 else 0 for n in shape)
    ref = F.conv_transpose3d(torch.from_numpy(x)[None], torch.from_numpy(W), torch.from_numpy(b),
                             stride=2, padding=1, output_padding=op)[0].numpy()
    np.testing.assert_allclose(nn.up(x, W, b, shape), ref, atol=1e-12)


def test_conv_adjoint_identity():
    x, W = rnd(7, 3, 5, 6, 4), rnd(8, 4, 3, 3, 3, 3)
    y = rnd(9, 4, 3, 3, 2)
    lhs = float((nn.conv(x, W, np.zeros(4), stride=2) * y).sum())
    rhs = float((x * nn.conv_adjoint(y, W, x.shape[1:], stride=2)).sum())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_parameter_count():
    # 3x3x3 convolutions with 16/32/64 channels, 4 inputs, 3 outputs:
    # weights enc0a..head, then biases (the two up layers output 32 and 16 channels)
    weights = 27 * (4 * 16 + 16 * 16 + 16 * 32 + 32 * 32 + 32 * 64 + 64 * 64
                    + 64 * 32 + 64 * 32 + 32 * 16 + 32 * 16) + 16 * 3
    biases = 16 + 16 + 32 + 32 + 64 + 64 + 32 + 32 + 16 + 16 + 3
    assert nn.n_params() == weights + biases == 354611


@pytest.mark.parametrize("mode", ["rel", "cos"])
def test_loss_gradient_matches_finite_differences(mode):
    ch = (2, 4, 6)
    shapes = nn.layer_shapes(ch)
    npar = nn.n_params(ch)
    rng = np.random.default_rng(11)
    blob = 0.3 * rng.standard_normal(npar)
    grid = (3, 4, 5)  # NZ, NY, NX
    rho = rng.uniform(0, 1, grid)
    r = rng.standard_normal(3 * int(np.prod(grid)))
    e = rng.standard_normal(r.size)
    fixed = np.zeros(r.size, bool)
    fixed[:6] = True
    r[fixed] = 0.0
    loss, g = nn.loss_and_grad(nn.unpack(blob, ch), rho, r, e, fixed, mode)
    gvec = np.concatenate([np.concatenate([g[n][0].ravel(), g[n][1].ravel()]) for n, _ in shapes])
    idx = rng.choice(npar, 60, replace=False)
    h = 1e-6
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (nn.loss_and_grad(nn.unpack(bp, ch), rho, r, e, fixed, mode)[0]
              - nn.loss_and_grad(nn.unpack(bm, ch), rho, r, e, fixed, mode)[0]) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gvec[i])


def test_node_density_averages_adjacent_elements():
    x = np.arange(24, dtype=float)  # nelx=4, nely=3, nelz=2
    rho = nn.node_density(x, 4, 3, 2)
    assert rho.shape == (3, 4, 5)
    assert rho[0, 0, 0] == 0.0  # corner node touches element 0 only
    # interior node (1,1,1) touches the 8 elements around it
    E = x.reshape(2, 3, 4)
    assert rho[1, 1, 1] == E[0:2, 0:2, 0:2].mean()


def test_cosine_loss_is_blind_to_positive_output_scale():
    # a network whose head is multiplied by c > 0 has the same loss; by -1, 2 - loss
    ch = (2, 4, 6)
    rng = np.random.default_rng(12)
    blob = 0.3 * rng.standard_normal(nn.n_params(ch))
    grid = (3, 4, 5)
    rho = rng.uniform(0, 1, grid)
    r = rng.standard_normal(3 * int(np.prod(grid)))
    e = rng.standard_normal(r.size)
    fixed = np.zeros(r.size, bool)
    P = nn.unpack(blob, ch)
    l1 = nn.loss_and_grad(P, rho, r, e, fixed, "cos")[0]
    Q = dict(P)
    Q["head"] = (P["head"][0] * 7.0, P["head"][1] * 7.0)
    l2 = nn.loss_and_grad(Q, rho, r, e, fixed, "cos")[0]
    Q["head"] = (-P["head"][0], -P["head"][1])
    l3 = nn.loss_and_grad(Q, rho, r, e, fixed, "cos")[0]
    assert 0.0 <= l1 <= 2.0 and abs(l1 - l2) < 1e-12 and abs(l1 + l3 - 2.0) < 1e-12
