"""FP64 oracle of the convolutional preconditioner network (test infrastructure).

The network maps four node fields -- the physical density averaged to the nodes
and the three residual components scaled by their root-mean-square -- to a
three-component correction on the same node grid.  It is a three-level
encoder-decoder of 3x3x3 convolutions:

  level 0: conv(4 -> c0), ReLU, conv(c0 -> c0), ReLU                 -> s0
  level 1: conv(c0 -> c1, stride 2), ReLU, conv(c1 -> c1), ReLU      -> s1
  level 2: conv(c1 -> c2, stride 2), ReLU, conv(c2 -> c2), ReLU
  up 1:    up(c2 -> c1) to the level-1 grid, concat [up, s1], conv(2 c1 -> c1), ReLU
  up 0:    up(c1 -> c0) to the level-0 grid, concat [up, s0], conv(2 c0 -> c0), ReLU
  head:    1x1x1 conv(c0 -> 3)

"conv" is zero-padded cross-correlation (padding 1 for 3x3x3, stride 1 or 2:
output size ceil(n / stride)); "up" is the transpose (adjoint) of the stride-2
3x3x3 convolution onto the finer grid, plus a bias.  Arrays are channel-first,
[C, D, H, W] with W the fastest axis (x), matching the node numbering.

Everything here is a plain loop over the 27 taps with NumPy slicing; the
backward pass is the exact adjoint of each step.  It shares nothing with the
HIP implementation.
"""

from __future__ import annotations

import numpy as np

CHANNELS = (16, 32, 64)


def layer_shapes(c=CHANNELS, cin=4, cout=3):
    """(name, weight shape, bias length) in the order the weight blob stores them."""
    c0, c1, c2 = c
    return [
        ("enc0a", (c0, cin, 3, 3, 3)), ("enc0b", (c0, c0, 3, 3, 3)),
        ("down1", (c1, c0, 3, 3, 3)), ("enc1b", (c1, c1, 3, 3, 3)),
        ("down2", (c2, c1, 3, 3, 3)), ("enc2b", (c2, c2, 3, 3, 3)),
        ("up1", (c2, c1, 3, 3, 3)), ("dec1", (c1, 2 * c1, 3, 3, 3)),
        ("up0", (c1, c0, 3, 3, 3)), ("dec0", (c0, 2 * c0, 3, 3, 3)),
        ("head", (cout, c0, 1, 1, 1)),
    ]


def bias_len(name, shape):
    # the up layers are transposes: weight [Cin_of_forward_conv..] -> output channels = shape[1]
    return shape[1] if name.startswith("up") else shape[0]


def n_params(c=CHANNELS):
    return sum(int(np.prod(s)) + bias_len(n, s) for n, s in layer_shapes(c))


def unpack(blob, c=CHANNELS):
    """Flat parameter vector -> dict name -> (W, b)."""
    out, o = {}, 0
    for name, shape in layer_shapes(c):
        nw = int(np.prod(shape))
        W = blob[o:o + nw].reshape(shape)
        o += nw
        nb = bias_len(name, shape)
        out[name] = (W, blob[o:o + nb])
        o += nb
    assert o == blob.size
    return out


def pack(params, c=CHANNELS):
    return np.concatenate([np.concatenate([params[n][0].ravel(), params[n][1].ravel()])
                           for n, _ in layer_shapes(c)])


# -- linear building blocks ---------------------------------------------------
def conv(x, W, b, stride=1):
    """Zero-padded cross-correlation; x [Ci, D, H, W], W [Co, Ci, k, k, k]."""
    k = W.shape[2]
    p = k // 2
    Ci, D, H, Wd = x.shape
    oD, oH, oW = (-(-D // stride), -(-H // stride), -(-Wd // stride))
    xp = np.zeros((Ci, D + 2 * p + stride, H + 2 * p + stride, Wd + 2 * p + stride))
    xp[:, p:p + D, p:p + H, p:p + Wd] = x
    out = np.zeros((W.shape[0], oD, oH, oW))
    for a in range(k):
        for bb in range(k):
            for c in range(k):
                xs = xp[:, a:a + stride * oD:stride, bb:bb + stride * oH:stride, c:c + stride * oW:stride]
                out += np.tensordot(W[:, :, a, bb, c], xs, axes=([1], [0]))
    return out + b[:, None, None, None]


def conv_adjoint(y, W, in_shape, stride=1):
    """Adjoint of conv without bias: maps [Co, oD, oH, oW] -> [Ci, *in_shape]."""
    k = W.shape[2]
    p = k // 2
    D, H, Wd = in_shape
    oD, oH, oW = y.shape[1:]
    xp = np.zeros((W.shape[1], D + 2 * p + stride, H + 2 * p + stride, Wd + 2 * p + stride))
    for a in range(k):
        for bb in range(k):
            for c in range(k):
                xp[:, a:a + stride * oD:stride, bb:bb + stride * oH:stride, c:c + stride * oW:stride] += \
                    np.tensordot(W[:, :, a, bb, c], y, axes=([0], [0]))
    return xp[:, p:p + D, p:p + H, p:p + Wd]


def conv_weight_grad(x, dy, k, stride=1):
    """dL/dW for conv given input x and output gradient dy."""
    p = k // 2
    Ci, D, H, Wd = x.shape
    oD, oH, oW = dy.shape[1:]
    xp = np.zeros((Ci, D + 2 * p + stride, H + 2 * p + stride, Wd + 2 * p + stride))
    xp[:, p:p + D, p:p + H, p:p + Wd] = x
    dW = np.zeros((dy.shape[0], Ci, k, k, k))
    for a in range(k):
        for bb in range(k):
            for c in range(k):
                xs = xp[:, a:a + stride * oD:stride, bb:bb + stride * oH:stride, c:c + stride * oW:stride]
                dW[:, :, a, bb, c] = np.tensordot(dy, xs, axes=([1, 2, 3], [1, 2, 3]))
    return dW


def up(x, W, b, out_shape):
    """Transpose of the stride-2 3x3x3 convolution onto out_shape, plus bias."""
    return conv_adjoint(x, W, out_shape, stride=2) + b[:, None, None, None]


def relu(x):
    return np.maximum(x, 0.0)


# -- network --------------------------------------------------------------------
def forward(params, x, keep=False):
    """x [4, D, H, W] -> out [3, D, H, W] (and the activations when keep)."""
    A = {"x": x}
    s = x.shape[1:]
    A["e0a"] = relu(conv(x, *params["enc0a"]))
    A["s0"] = relu(conv(A["e0a"], *params["enc0b"]))
    A["d1"] = relu(conv(A["s0"], *params["down1"], stride=2))
    A["s1"] = relu(conv(A["d1"], *params["enc1b"]))
    A["d2"] = relu(conv(A["s1"], *params["down2"], stride=2))
    A["b2"] = relu(conv(A["d2"], *params["enc2b"]))
    A["u1"] = up(A["b2"], *params["up1"], A["s1"].shape[1:])
    A["c1"] = np.concatenate([A["u1"], A["s1"]])
    A["t1"] = relu(conv(A["c1"], *params["dec1"]))
    A["u0"] = up(A["t1"], *params["up0"], s)
    A["c0"] = np.concatenate([A["u0"], A["s0"]])
    A["t0"] = relu(conv(A["c0"], *params["dec0"]))
    out = conv(A["t0"], *params["head"])
    return (out, A) if keep else out


def backward(params, A, dout):
    """Gradients of a scalar loss with dL/dout = dout; returns dict like params."""
    g = {}

    def conv_back(name, x, y, dy, stride=1, act=True):
        W, _ = params[name]
        if act:
            dy = dy * (y > 0)
        g[name] = (conv_weight_grad(x, dy, W.shape[2], stride), dy.sum(axis=(1, 2, 3)))
        return conv_adjoint(dy, W, x.shape[1:], stride)

    def up_back(name, x, dy):
        W, _ = params[name]
        # y = conv_s2^T(x; W): dL/dx = conv_s2(dy; W), dL/dW from the forward pairing
        g[name] = (conv_weight_grad(dy, x, 3, stride=2), dy.sum(axis=(1, 2, 3)))
        return conv(dy, W, np.zeros(W.shape[0]), stride=2)

    dt0 = conv_back("head", A["t0"], None, dout, act=False)
    dc0 = conv_back("dec0", A["c0"], A["t0"], dt0)
    c0 = params["up0"][0].shape[1]
    du0, ds0 = dc0[:c0], dc0[c0:]
    dt1 = up_back("up0", A["t1"], du0)
    dc1 = conv_back("dec1", A["c1"], A["t1"], dt1)
    c1 = params["up1"][0].shape[1]
    du1, ds1 = dc1[:c1], dc1[c1:]
    db2 = up_back("up1", A["b2"], du1)
    dd2 = conv_back("enc2b", A["d2"], A["b2"], db2)
    ds1 = ds1 + conv_back("down2", A["s1"], A["d2"], dd2, stride=2)
    dd1 = conv_back("enc1b", A["d1"], A["s1"], ds1)
    ds0 = ds0 + conv_back("down1", A["s0"], A["d1"], dd1, stride=2)
    de0a = conv_back("enc0b", A["e0a"], A["s0"], ds0)
    conv_back("enc0a", A["x"], A["e0a"], de0a)
    return g


# -- preconditioner inputs / outputs and loss -----------------------------------
def node_density(xphys, nelx, nely, nelz):
    """Mean of the elements around each node -> [NZ, NY, NX]."""
    E = xphys.reshape(nelz, nely, nelx)
    acc = np.zeros((nelz + 1, nely + 1, nelx + 1))
    cnt = np.zeros_like(acc)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                acc[dz:dz + nelz, dy:dy + nely, dx:dx + nelx] += E
                cnt[dz:dz + nelz, dy:dy + nely, dx:dx + nelx] += 1
    return acc / cnt


def rms(v):
    return float(np.sqrt(np.mean(v * v)))


def make_input(rho_node, r):
    """[4, NZ, NY, NX]: density and residual / rms(residual)."""
    s = rms(r)
    R = (r / s).reshape(rho_node.shape + (3,))
    return np.concatenate([rho_node[None], np.moveaxis(R, -1, 0)]), s


def apply(params, rho_node, r, fixed_mask):
    """z = rms(r) * net(rho, r / rms(r)), zero on fixed dofs."""
    x, s = make_input(rho_node, r)
    out = forward(params, x)
    z = s * np.moveaxis(out, 0, -1).reshape(-1)
    z[fixed_mask] = 0.0
    return z


def loss_and_grad(params, rho_node, r, e, fixed_mask, mode="rel"):
    """Loss of the scaled prediction y = net(rho, r/s) against t = e/s (s = rms(r)),
    over the free dofs, and its parameter gradient.

    mode "rel":    ||y - t||^2 / ||t||^2 (relative squared error);
    mode "cos":    1 - y.t / (|y| |t|) (one minus the cosine of the angle), blind to
                   a positive scaling of y (so is flexible CG) but not to its sign.
    """
    x, s = make_input(rho_node, r)
    out, A = forward(params, x, keep=True)
    t = np.moveaxis((e / s).reshape(rho_node.shape + (3,)), -1, 0)
    m = np.moveaxis((~fixed_mask).reshape(rho_node.shape + (3,)), -1, 0).astype(float)
    tm = t * m
    den = float((tm * tm).sum())
    if mode == "rel":
        diff = (out - t) * m
        loss = float((diff * diff).sum()) / den
        dout = 2.0 * diff / den
    elif mode == "cos":
        ym = out * m
        a = float((ym * tm).sum())
        b = float((ym * ym).sum())
        q = np.sqrt(b * den)
        loss = 1.0 - a / q
        dout = (a / b * ym - tm) / q
    else:
        raise ValueError(mode)
    g = backward(params, A, dout)
    return loss, g
