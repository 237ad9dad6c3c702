"""Seeded parameters and inputs for the convolutional preconditioner network
(random draws and the blob layout only; no network arithmetic).

Blob layout: per layer the weight [c_out, c_in, k, k, k] (row-major) followed by
its bias, layers in the order of ``layer_shapes``.  The two up layers store the
weight of the stride-2 convolution they transpose, [c_coarse, c_fine, 3, 3, 3],
and a bias of c_fine entries.
"""

from __future__ import annotations

import numpy as np

CHANNELS = (16, 32, 64)


def layer_shapes(c=CHANNELS, cin: int = 4, cout: int = 3):
    """[(name, weight shape, bias length)] in blob order."""
    c0, c1, c2 = c
    k = (3, 3, 3)
    return [
        ("enc0a", (c0, cin) + k, c0), ("enc0b", (c0, c0) + k, c0),
        ("down1", (c1, c0) + k, c1), ("enc1b", (c1, c1) + k, c1),
        ("down2", (c2, c1) + k, c2), ("enc2b", (c2, c2) + k, c2),
        ("up1", (c2, c1) + k, c1), ("dec1", (c1, 2 * c1) + k, c1),
        ("up0", (c1, c0) + k, c0), ("dec0", (c0, 2 * c0) + k, c0),
        ("head", (cout, c0, 1, 1, 1), cout),
    ]


def n_params(c=CHANNELS) -> int:
    return sum(int(np.prod(w)) + b for _, w, b in layer_shapes(c))


def init_weights(c=CHANNELS, seed: int = 0, bias_scale: float = 0.05) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in), fan_in = prod(shape[1:]); for
    an up layer the fan-in of a fine point is c_coarse * 27 / 8) and uniform
    biases in [-bias_scale, bias_scale]; float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, w, nb in layer_shapes(c):
        fan = w[0] * 27 / 8 if name.startswith("up") else int(np.prod(w[1:]))
        bound = np.sqrt(6.0 / fan)
        parts.append(rng.uniform(-bound, bound, int(np.prod(w))))
        parts.append(rng.uniform(-bias_scale, bias_scale, nb))
    return np.concatenate(parts).astype(np.float32)


def random_activations(seed: int, channels: int, batch: int, nodes) -> np.ndarray:
    """[channels, batch, NZ, NY, NX] standard-normal field (float32); channel 0
    is drawn uniform in [0, 1] like a density."""
    nx, ny, nz = nodes
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((channels, batch, nz, ny, nx))
    x[0] = rng.uniform(0.0, 1.0, (batch, nz, ny, nx))
    return x.astype(np.float32)
