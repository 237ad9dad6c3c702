"""Optimality Criteria update with move limits and a volume multiplier
(Optimality Criteria section).

For a multiplier lambda > 0 every design element j moves to

    x_new_j = clamp( x_j * (max(0, -dc_j) / (lambda dv_j))^eta ,
                     max(0, x_j - move), min(1, x_j + move) )

(passive elements keep their value; the max(0, .) only guards against a
rounding-negative energy).  The volume measure V(x_new) is non-increasing in
lambda; the update takes the lambda at which it meets the target V*.

Two ways of finding lambda are given:

* ``oc_bisection`` -- the classic bisection: bracket [0, 1e9], arithmetic
  midpoint, move the lower end up when the volume at the midpoint is above the
  target, stop when (l2 - l1)/(l1 + l2) < tol, return the design at the last
  midpoint.  The volume is evaluated by its plain definition (for the density
  filter: filter the candidate design and sum the physical densities of design
  elements), i.e. the filter runs inside the search loop.
* ``oc_exact`` -- the exact root of the piecewise-power function
  V(lambda) = A + B lambda^(-eta) between consecutive breakpoints at which an
  element hits one of its bounds, using the linear volume weights w.
"""

from __future__ import annotations

import numpy as np


def oc_candidate(x, dc, dv, lam, move, eta, design):
    """x_new(lambda) for all elements (passive ones unchanged)."""
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)
    with np.errstate(divide="ignore", invalid="ignore"):
        B = np.maximum(0.0, -dc) / (lam * dv)
        cand = x * B ** eta
    xn = np.minimum(hi, np.maximum(lo, cand))
    return np.where(design, xn, x)


def oc_bisection(x, dc, dv, volume_of, target, move=0.2, eta=0.5, design=None, tol=1e-12,
                 l1=0.0, l2=1e9, max_steps=400):
    """Bisection on lambda; ``volume_of(xnew)`` is the plain volume measure."""
    design = np.ones(x.shape, dtype=bool) if design is None else design
    xnew, mid = x.copy(), 0.5 * (l1 + l2)
    steps = 0
    while (l2 - l1) / (l1 + l2) > tol and steps < max_steps:
        mid = 0.5 * (l1 + l2)
        xnew = oc_candidate(x, dc, dv, mid, move, eta, design)
        if volume_of(xnew) > target:
            l1 = mid
        else:
            l2 = mid
        steps += 1
    return xnew, mid, (l1, l2)


def oc_exact(x, dc, dv, w, target, move=0.2, eta=0.5, design=None):
    """Exact multiplier for V(x) = w^T x (w >= 0).  Returns (x_new, lambda)."""
    design = np.ones(x.shape, dtype=bool) if design is None else design
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)
    a = np.zeros_like(x)
    d = design
    a[d] = x[d] * (np.maximum(0.0, -dc[d]) / dv[d]) ** eta
    const = float(w[~d] @ x[~d])
    # element j: x = hi for lam <= lh_j, a lam^-eta between, lo for lam >= ll_j
    with np.errstate(divide="ignore"):
        lh = np.where(a > 0, (a / hi) ** (1.0 / eta), 0.0)
        ll = np.where((a > 0) & (lo > 0), (a / np.where(lo > 0, lo, 1.0)) ** (1.0 / eta), np.inf)
    lh = np.where(d, lh, 0.0)
    ll = np.where(d, ll, np.inf)

    def V(lam):
        return float(w @ oc_candidate(x, dc, dv, lam, move, eta, design))

    bps = np.unique(np.concatenate([lh[d & (a > 0)], ll[d & np.isfinite(ll)]]))
    bps = bps[bps > 0]
    if bps.size == 0:
        return oc_candidate(x, dc, dv, 1.0, move, eta, design), 1.0
    # V is non-increasing in lambda: binary search over the sorted breakpoints
    if V(bps[0]) <= target:
        # already at or below the target at the smallest breakpoint: every element
        # is at its upper bound or at a flat lower part; any lambda below works
        lam = bps[0] * 0.5
        return oc_candidate(x, dc, dv, lam, move, eta, design), lam
    if V(bps[-1]) >= target:
        lam = bps[-1] * 2.0
        return oc_candidate(x, dc, dv, lam, move, eta, design), lam
    # first breakpoint with V <= target; root lies in (bps[k-1], bps[k]]
    lo_k, hi_k = 0, bps.size - 1          # V(bps[lo_k]) > target >= V(bps[hi_k])
    while hi_k - lo_k > 1:
        m = (lo_k + hi_k) // 2
        if V(bps[m]) > target:
            lo_k = m
        else:
            hi_k = m
    k = hi_k
    lamL, lamR = bps[k - 1], bps[k]
    mid = 0.5 * (lamL + lamR)
    between = d & (lh <= lamL) & (ll >= lamR) & (a > 0)
    at_hi = d & (lh >= lamR)
    at_lo = d & ~between & ~at_hi
    A = const + float(w[at_hi] @ hi[at_hi]) + float(w[at_lo] @ lo[at_lo])
    Bc = float(w[between] @ a[between])
    if Bc <= 0.0 or target <= A:
        lam = mid
    else:
        lam = (Bc / (target - A)) ** (1.0 / eta)
        lam = min(max(lam, lamL), lamR)
    return oc_candidate(x, dc, dv, lam, move, eta, design), lam
