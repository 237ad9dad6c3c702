"""Cone-weight spatial filter (Sensitivity Filtering section).

H_ei = max(0, rmin - |c_e - c_i|) over element centroids (unit element size,
rmin in element units), truncated at the domain boundary; Hs_e = sum_i H_ei.

Applications (readings of the filter statement, which prints dc~ = H dc without
its normalisation):

* density filter, forward:   xPhys = (H x) / Hs, then passive elements reset to
  their fixed value;
* density filter, adjoint:   dx = H (g / Hs) where g is the gradient with respect
  to xPhys restricted to design elements (the passive reset has zero derivative);
* sensitivity filter:        dc~ = H (x * dc) / (Hs * max(gamma, x)), gamma = 1e-3;
* filtered volume weights:   w^D = H (1_D / Hs), so that the design-element sum of
  xPhys equals (w^D)^T x.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

SENS_GAMMA = 1e-3


def filter_offsets(rmin: float):
    """Integer offsets d with |d| < rmin and their weights rmin - |d|."""
    r = int(math.ceil(rmin)) - 1
    offs, wts = [], []
    for dk in range(-r, r + 1):
        for dj in range(-r, r + 1):
            for di in range(-r, r + 1):
                dist = math.sqrt(di * di + dj * dj + dk * dk)
                if dist < rmin:
                    offs.append((di, dj, dk))
                    wts.append(rmin - dist)
    return offs, wts


def filter_matrix(nelx: int, nely: int, nelz: int, rmin: float) -> sp.csr_matrix:
    """Sparse H by enumerating, for every element, the neighbours inside rmin."""
    nel = nelx * nely * nelz
    offs, wts = filter_offsets(rmin)
    e = np.arange(nel)
    i = e % nelx
    j = (e // nelx) % nely
    k = e // (nelx * nely)
    rows, cols, vals = [], [], []
    for (di, dj, dk), w in zip(offs, wts):
        ii, jj, kk = i + di, j + dj, k + dk
        ok = (ii >= 0) & (ii < nelx) & (jj >= 0) & (jj < nely) & (kk >= 0) & (kk < nelz)
        rows.append(e[ok])
        cols.append((ii + nelx * (jj + nely * kk))[ok])
        vals.append(np.full(int(ok.sum()), w))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nel, nel)).tocsr()


def filter_rows(nelx, nely, nelz, rmin, elems):
    """For selected elements: list of (neighbour indices, weights) of their H rows."""
    offs, wts = filter_offsets(rmin)
    rows = []
    for e in np.asarray(elems):
        i, j, k = e % nelx, (e // nelx) % nely, e // (nelx * nely)
        idx, w = [], []
        for (di, dj, dk), wt in zip(offs, wts):
            ii, jj, kk = i + di, j + dj, k + dk
            if 0 <= ii < nelx and 0 <= jj < nely and 0 <= kk < nelz:
                idx.append(ii + nelx * (jj + nely * kk))
                w.append(wt)
        rows.append((np.array(idx), np.array(w)))
    return rows


def filter_matrix_bruteforce(nelx: int, nely: int, nelz: int, rmin: float) -> np.ndarray:
    """Dense H from all centroid pairs (tiny grids only)."""
    e = np.arange(nelx * nely * nelz)
    c = np.stack([e % nelx, (e // nelx) % nely, e // (nelx * nely)], axis=1).astype(float) + 0.5
    d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
    return np.maximum(0.0, rmin - d)


class Filter:
    """H, Hs and the passive mask of one problem."""

    def __init__(self, nelx, nely, nelz, rmin, mask=None):
        self.H = filter_matrix(nelx, nely, nelz, rmin)
        self.Hs = np.asarray(self.H.sum(axis=1)).ravel()
        nel = nelx * nely * nelz
        self.mask = np.zeros(nel, dtype=np.int8) if mask is None else np.asarray(mask, np.int8)
        self.design = self.mask == 0

    def forward(self, x: np.ndarray) -> np.ndarray:
        xp = (self.H @ x) / self.Hs
        xp[self.mask == 1] = 0.0
        xp[self.mask == 2] = 1.0
        return xp

    def adjoint(self, g: np.ndarray) -> np.ndarray:
        return self.H @ (np.where(self.design, g, 0.0) / self.Hs)

    def sensitivity(self, x: np.ndarray, dc: np.ndarray) -> np.ndarray:
        return (self.H @ (x * dc)) / (self.Hs * np.maximum(SENS_GAMMA, x))

    def volume_weights(self) -> np.ndarray:
        return self.H @ (self.design.astype(float) / self.Hs)
