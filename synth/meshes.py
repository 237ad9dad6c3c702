"""Seeded closed triangle meshes for the STL design-domain path (vertex and
triangle generation only): an axis-aligned box and a subdivided icosahedron
projected onto a sphere.  Triangles are (n, 3, 3) float32 arrays, counter-
clockwise seen from outside."""

from __future__ import annotations

import numpy as np


def box_mesh(lo, hi) -> np.ndarray:
    """12 triangles of the box [lo, hi] (3-vectors)."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    c = np.array([[lo[0] if (b >> 0) & 1 == 0 else hi[0], lo[1] if (b >> 1) & 1 == 0 else hi[1],
                   lo[2] if (b >> 2) & 1 == 0 else hi[2]] for b in range(8)])
    # corner index b = x + 2y + 4z; quads counter-clockwise seen from outside
    quads = [(0, 4, 6, 2), (1, 3, 7, 5), (0, 1, 5, 4), (2, 6, 7, 3), (0, 2, 3, 1), (4, 5, 7, 6)]
    tri = []
    for a, b, cc, d in quads:
        tri += [(c[a], c[b], c[cc]), (c[a], c[cc], c[d])]
    return np.array(tri, dtype=np.float32)


def sphere_mesh(center, radius, subdivisions=3) -> np.ndarray:
    """Icosahedron subdivided `subdivisions` times, vertices on the sphere."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, float) / np.linalg.norm(p) for p in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdivisions):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                mid[key] = len(v) - 1
            return mid[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    V = np.asarray(center, float) + radius * np.array(v)
    return V[np.array(f)].astype(np.float32)


def random_voxels(seed, dims, fill=0.35) -> np.ndarray:
    """Random 0/1 element field (a density already thresholded), float64."""
    rng = np.random.default_rng(seed)
    return (rng.random(int(np.prod(dims))) < fill).astype(np.float64)
