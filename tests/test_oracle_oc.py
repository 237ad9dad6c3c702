"""Pins of the oracle's OC update and volume multiplier (Optimality Criteria section)."""

import numpy as np
import pytest

import synth
from oracle import filt, oc


def setup_case(seed, nel=400, passive=True):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, nel)
    x[rng.random(nel) < 0.1] = 0.0
    dc = -rng.exponential(1.0, nel) * rng.uniform(0, 3, nel) ** 2
    dv = rng.uniform(0.5, 1.5, nel)
    design = np.ones(nel, bool)
    if passive:
        design[rng.random(nel) < 0.1] = False
    w = dv.copy()
    return x, dc, dv, w, design


@pytest.mark.parametrize("seed", range(5))
def test_exact_root_meets_target_and_equals_bisection(seed):
    x, dc, dv, w, design = setup_case(seed)
    target = float(w @ x)  # keep the current volume
    xe, lam = oc.oc_exact(x, dc, dv, w, target, 0.2, 0.5, design)
    assert abs(w @ xe - target) < 1e-11 * target
    xb, lb, (l1, l2) = oc.oc_bisection(x, dc, dv, lambda z: float(w @ z), target, 0.2, 0.5,
                                       design, tol=1e-13)
    assert abs(lb - lam) <= 1e-11 * lam
    np.testing.assert_allclose(xb, xe, atol=1e-10)
    # bracket at exit
    vol = lambda lmb: float(w @ oc.oc_candidate(x, dc, dv, lmb, 0.2, 0.5, design))
    assert vol(l2) <= target <= vol(l1)


def test_move_and_box_limits_and_passive():
    x, dc, dv, w, design = setup_case(11)
    xe, _ = oc.oc_exact(x, dc, dv, w, 0.8 * float(w @ x), 0.15, 0.5, design)
    assert np.all(xe >= 0) and np.all(xe <= 1)
    assert np.all(np.abs(xe - x) <= 0.15 + 1e-15)
    assert np.array_equal(xe[~design], x[~design])


def test_kkt_point_is_fixed_point():
    """dc = -lam0 dv on every design element: at lam0 the OC factor is 1, so the
    design is a fixed point when it already meets the volume target."""
    rng = np.random.default_rng(3)
    nel = 300
    x = rng.uniform(0.3, 0.7, nel)
    dv = rng.uniform(0.5, 1.5, nel)
    lam0 = 2.7
    dc = -lam0 * dv
    design = np.ones(nel, bool)
    xe, lam = oc.oc_exact(x, dc, dv, dv, float(dv @ x), 0.2, 0.5, design)
    assert abs(lam - lam0) < 1e-12 * lam0
    np.testing.assert_allclose(xe, x, atol=1e-14)


def test_density_filter_bisection_runs_filter_inside_loop():
    """Plain bisection with the filter applied to every candidate agrees with the
    exact root computed from the linear filtered-volume weights."""
    p = synth.config_obstacle(seed=5)
    F = filt.Filter(p.nelx, p.nely, p.nelz, p.rmin, p.mask)
    design = p.mask == 0
    x = p.initial_design()
    rng = np.random.default_rng(9)
    dc = -rng.exponential(1.0, p.nel)
    dcf = F.adjoint(dc)
    w = F.volume_weights()
    target = p.volfrac * design.sum()
    xe, lam = oc.oc_exact(x, dcf, w, w, target, p.move, p.eta, design)
    xb, lb, _ = oc.oc_bisection(x, dcf, w, lambda z: float(F.forward(z)[design].sum()), target,
                                p.move, p.eta, design, tol=1e-12)
    assert abs(lb - lam) <= 3e-12 * lam
    np.testing.assert_allclose(xb, xe, atol=1e-9)
    assert abs(F.forward(xe)[design].sum() - target) < 1e-8
