"""Seeded cantilever-type problem instances (inputs only, no method arithmetic)."""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

DESIGN, VOID, SOLID = 0, 1, 2


@dataclasses.dataclass
class Problem:
    """One SIMP compliance problem: grid, material, optimiser constants, BCs, load.

    ``mask`` has ``nel`` int8 entries (0 design, 1 void, 2 solid),
    ``fixed_dofs`` lists constrained degrees of freedom (homogeneous Dirichlet),
    ``f`` is the nodal load vector of length ``ndof`` (dof = 3*node + c).
    """

    nelx: int
    nely: int
    nelz: int
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    penal: float = 3.0
    rmin: float = 1.5
    volfrac: float = 0.3
    move: float = 0.2
    eta: float = 0.5
    mask: Optional[np.ndarray] = None
    fixed_dofs: Optional[np.ndarray] = None
    f: Optional[np.ndarray] = None
    n_iter: int = 10
    filter_mode: str = "density"  # "density" | "sensitivity"
    vol_mode: str = "design"  # volume target over "design" elements or "all" elements
    name: str = ""
    seed: int = 0

    @property
    def nel(self) -> int:
        return self.nelx * self.nely * self.nelz

    @property
    def nnodes(self) -> int:
        return (self.nelx + 1) * (self.nely + 1) * (self.nelz + 1)

    @property
    def ndof(self) -> int:
        return 3 * self.nnodes

    def node_id(self, i, j, k):
        return np.asarray(i) + (self.nelx + 1) * (np.asarray(j) + (self.nely + 1) * np.asarray(k))

    def elem_id(self, i, j, k):
        return np.asarray(i) + self.nelx * (np.asarray(j) + self.nely * np.asarray(k))

    def initial_design(self) -> np.ndarray:
        """x0: ``volfrac`` on design elements, 0 on void, 1 on solid elements."""
        x = np.full(self.nel, float(self.volfrac))
        if self.mask is not None:
            x[self.mask == VOID] = 0.0
            x[self.mask == SOLID] = 1.0
        return x

    def describe(self) -> dict:
        return {
            "name": self.name,
            "grid": [self.nelx, self.nely, self.nelz],
            "nel": self.nel,
            "ndof": self.ndof,
            "free_dof": int(self.ndof - len(self.fixed_dofs)),
            "rmin": self.rmin,
            "volfrac": self.volfrac,
            "penal": self.penal,
            "n_iter": self.n_iter,
            "seed": self.seed,
        }


def _face_nodes(p: Problem, axis: int, side: int):
    """Node indices on the face ``axis``-coordinate == 0 (side 0) or == n (side 1)."""
    n = [p.nelx, p.nely, p.nelz]
    rng = [np.arange(m + 1) for m in n]
    rng[axis] = np.array([0 if side == 0 else n[axis]])
    I, J, K = np.meshgrid(rng[0], rng[1], rng[2], indexing="ij")
    return p.node_id(I.ravel(), J.ravel(), K.ravel())


def _clamp_face(p: Problem, axis: int, side: int) -> np.ndarray:
    nodes = _face_nodes(p, axis, side)
    return np.sort((3 * nodes[:, None] + np.arange(3)[None, :]).ravel()).astype(np.int64)


def cantilever(nelx, nely, nelz, *, volfrac, rmin, n_iter, penal=3.0, E0=1.0, Emin=1e-9,
               nu=0.3, move=0.2, eta=0.5, name="cantilever", seed=0) -> Problem:
    """Cantilever: face x=0 clamped; total load -1 in y spread equally over the
    nodes of the bottom edge (j=0) at the free end x=nelx."""
    p = Problem(nelx, nely, nelz, E0=E0, Emin=Emin, nu=nu, penal=penal, rmin=rmin,
                volfrac=volfrac, move=move, eta=eta, n_iter=n_iter, name=name, seed=seed)
    p.mask = np.zeros(p.nel, dtype=np.int8)
    p.fixed_dofs = _clamp_face(p, 0, 0)
    f = np.zeros(p.ndof)
    k = np.arange(nelz + 1)
    loaded = p.node_id(nelx, 0, k)
    f[3 * loaded + 1] = -1.0 / (nelz + 1)
    p.f = f
    return p


def config_small() -> Problem:
    """20x10x4 cantilever, rmin 1.5, volfrac 0.3, 10 OC iterations (3465 DOF)."""
    return cantilever(20, 10, 4, volfrac=0.3, rmin=1.5, n_iter=10, name="cantilever-20x10x4")


def _eligible_for_mask(p: Problem) -> np.ndarray:
    """Elements a random mask may touch: not in the clamped layer (i = 0) and not
    adjacent to the loaded bottom edge of the free end."""
    e = np.arange(p.nel)
    i = e % p.nelx
    j = (e // p.nelx) % p.nely
    return (i >= 1) & ~((i == p.nelx - 1) & (j == 0))


def config_obstacle(seed: int = 2) -> Problem:
    """60x30x20 cantilever with a seeded passive-void box covering a fraction
    U[0.05, 0.15] of the voxels plus a Bernoulli(0.1) void mask over the remaining
    eligible design elements; rmin 2.0, volfrac 0.25, 50 OC iterations."""
    p = cantilever(60, 30, 20, volfrac=0.25, rmin=2.0, n_iter=50,
                   name="cantilever-obstacle-60x30x20", seed=seed)
    rng = np.random.default_rng(seed)
    frac = rng.uniform(0.05, 0.15)
    dims = np.array([p.nelx, p.nely, p.nelz], dtype=float)
    aspect = rng.uniform(0.7, 1.3, size=3)
    side = dims * (frac ** (1.0 / 3.0)) * aspect / np.prod(aspect) ** (1.0 / 3.0)
    side = np.clip(np.round(side).astype(int), 1, (dims - 4).astype(int))
    lo = [int(rng.integers(2, p.nelx - 2 - side[0] + 1)),
          int(rng.integers(1, p.nely - side[1] + 1)),
          int(rng.integers(0, p.nelz - side[2] + 1))]
    e = np.arange(p.nel)
    i = e % p.nelx
    j = (e // p.nelx) % p.nely
    k = e // (p.nelx * p.nely)
    inbox = ((i >= lo[0]) & (i < lo[0] + side[0]) & (j >= lo[1]) & (j < lo[1] + side[1])
             & (k >= lo[2]) & (k < lo[2] + side[2]))
    elig = _eligible_for_mask(p)
    mask = np.zeros(p.nel, dtype=np.int8)
    mask[inbox & elig] = VOID
    rest = elig & (mask == DESIGN)
    mask[rest & (rng.random(p.nel) < 0.1)] = VOID
    p.mask = mask
    return p


def config_large() -> Problem:
    """160x80x80 cantilever (3,168,963 DOF), rmin 3.0, volfrac 0.2, 30 OC iterations."""
    return cantilever(160, 80, 80, volfrac=0.2, rmin=3.0, n_iter=30, name="cantilever-160x80x80")


def config_paper_benchmark() -> Problem:
    """The paper's timed workload (Performance Comparison section): 32x16x16,
    volfrac 0.2, penal 3, rmin 4.0, 200 iterations; face x=0 clamped, a unit
    downward point load at the centre of the free end's bottom edge."""
    p = cantilever(32, 16, 16, volfrac=0.2, rmin=4.0, n_iter=200, name="paper-benchmark-32x16x16")
    f = np.zeros(p.ndof)
    f[3 * int(p.node_id(32, 0, 8)) + 1] = -1.0
    p.f = f
    return p


def random_problem(seed: int, nelx: Optional[int] = None, *, n_iter: int = 30,
                   boxes: Optional[int] = None) -> Problem:
    """Random cantilever-like problem: a random clamped face, a point load of unit
    magnitude in a uniformly random direction at a random node of the opposite
    face, 0-2 passive void boxes of 1-5 % of the voxels each, volfrac U[0.2, 0.4],
    rmin U[1.5, 3.0].  Grid ``nelx = 8*U{3..12}``, ``nely = nelz = nelx/2``."""
    rng = np.random.default_rng(seed)
    if nelx is None:
        nelx = 8 * int(rng.integers(3, 13))
    nely = nelz = nelx // 2
    volfrac = float(rng.uniform(0.2, 0.4))
    rmin = float(rng.uniform(1.5, 3.0))
    p = Problem(nelx, nely, nelz, volfrac=volfrac, rmin=rmin, n_iter=n_iter,
                name=f"random-{nelx}x{nely}x{nelz}-s{seed}", seed=seed)
    axis = int(rng.integers(0, 3))
    side = int(rng.integers(0, 2))
    p.fixed_dofs = _clamp_face(p, axis, side)
    n = [nelx, nely, nelz]
    load_ijk = [int(rng.integers(0, m + 1)) for m in n]
    load_ijk[axis] = n[axis] if side == 0 else 0
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    f = np.zeros(p.ndof)
    ln = int(p.node_id(*load_ijk))
    f[3 * ln:3 * ln + 3] = d
    p.f = f
    # passive boxes avoid the clamped layer and the elements around the load node
    e = np.arange(p.nel)
    ijk = [e % nelx, (e // nelx) % nely, e // (nelx * nely)]
    clamp_layer = ijk[axis] == (0 if side == 0 else n[axis] - 1)
    near_load = np.ones(p.nel, dtype=bool)
    for a in range(3):
        near_load &= (ijk[a] >= load_ijk[a] - 1) & (ijk[a] <= load_ijk[a])
    elig = ~clamp_layer & ~near_load
    mask = np.zeros(p.nel, dtype=np.int8)
    nb = int(rng.integers(0, 3)) if boxes is None else boxes
    for _ in range(nb):
        frac = rng.uniform(0.01, 0.05)
        s = np.maximum(1, np.round(np.array(n) * frac ** (1.0 / 3.0)).astype(int))
        lo = [int(rng.integers(0, n[a] - s[a] + 1)) for a in range(3)]
        inbox = np.ones(p.nel, dtype=bool)
        for a in range(3):
            inbox &= (ijk[a] >= lo[a]) & (ijk[a] < lo[a] + s[a])
        mask[inbox & elig] = VOID
    p.mask = mask
    return p


def batch_problems(n: int = 64, *, n_iter: int = 30, first_seed: int = 0) -> List[Problem]:
    """``n`` independent random problems of uneven sizes (seeds first_seed..)."""
    return [random_problem(first_seed + s, n_iter=n_iter) for s in range(n)]


def random_vector(seed: int, n: int, scale: float = 1.0) -> np.ndarray:
    """Standard-normal FP64 vector of length ``n``."""
    return scale * np.random.default_rng(seed).standard_normal(n)


def random_density(seed: int, nel: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform densities in [lo, hi]."""
    return np.random.default_rng(seed).uniform(lo, hi, size=nel)
