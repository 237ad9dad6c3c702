"""Pins of the oracle's cone-weight filter (Sensitivity Filtering section)."""

import math

import numpy as np
import pytest

import synth
from oracle import filt

# Interior row sums Hs = sum over lattice offsets |d| < rmin of (rmin - |d|),
# counted by hand in shells of equal |d|^2 (number of integer points per shell):
# |d|^2: 0:1 1:6 2:12 3:8 4:6 5:24 6:24 8:12 9:30 10:24 11:24 12:8 13:24 14:48
SHELLS = {0: 1, 1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24, 8: 12, 9: 30, 10: 24, 11: 24,
          12: 8, 13: 24, 14: 48}


def golden_hs():
    rows = {}
    with open("tests/golden/filter_interior_rowsum.txt") as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                r, npts, hs = line.split()
                rows[float(r)] = (int(npts), float(hs))
    return rows


@pytest.mark.parametrize("rmin", [1.5, 2.0, 3.0, 4.0])
def test_interior_rowsum_and_count(rmin):
    n = 2 * int(math.ceil(rmin)) + 1
    H = filt.filter_matrix(n, n, n, rmin)
    centre = (n // 2) * (1 + n + n * n)
    row = H.getrow(centre)
    shells = sum(cnt * (rmin - math.sqrt(s)) for s, cnt in SHELLS.items() if math.sqrt(s) < rmin)
    npts, hs = golden_hs()[rmin]
    assert row.nnz == npts == sum(c for s, c in SHELLS.items() if math.sqrt(s) < rmin)
    assert abs(row.sum() - shells) < 1e-12
    assert abs(row.sum() - hs) < 1e-6


@pytest.mark.parametrize("dims,rmin", [((5, 4, 3), 1.5), ((6, 3, 4), 2.0), ((7, 5, 4), 3.0), ((5, 5, 5), 4.0)])
def test_stencil_matrix_equals_bruteforce(dims, rmin):
    H = filt.filter_matrix(*dims, rmin).toarray()
    np.testing.assert_allclose(H, filt.filter_matrix_bruteforce(*dims, rmin), atol=1e-14)
    np.testing.assert_allclose(H, H.T, atol=0)


def test_forward_preserves_constants_and_partition_of_unity():
    F = filt.Filter(9, 6, 5, 2.0)
    np.testing.assert_allclose(F.forward(np.full(270, 0.37)), 0.37, rtol=1e-14)
    Hd = F.H.toarray()
    np.testing.assert_allclose((Hd / F.Hs[:, None]).sum(1), 1.0, rtol=1e-14)


def test_adjoint_identity_with_passive_elements():
    p = synth.config_obstacle(seed=3)
    F = filt.Filter(p.nelx, p.nely, p.nelz, p.rmin, p.mask)
    a = synth.random_vector(1, p.nel)
    b = synth.random_vector(2, p.nel)
    design = p.mask == 0
    lhs = float(F.forward(a)[design] @ b[design])
    rhs = float(a @ F.adjoint(b))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_filtered_volume_identity():
    p = synth.config_obstacle(seed=4)
    F = filt.Filter(p.nelx, p.nely, p.nelz, p.rmin, p.mask)
    x = p.initial_design()
    x[p.mask == 0] = synth.random_density(7, int((p.mask == 0).sum()))
    w = F.volume_weights()
    assert abs(F.forward(x)[p.mask == 0].sum() - w @ x) < 1e-9
    assert np.all(F.forward(x)[p.mask == 1] == 0.0)


def test_sensitivity_filter_of_uniform_field():
    # uniform x and uniform dc: H(x dc)/(Hs x) = dc exactly
    F = filt.Filter(6, 5, 4, 1.5)
    np.testing.assert_allclose(F.sensitivity(np.full(120, 0.5), np.full(120, -2.0)), -2.0, rtol=1e-14)


def test_sampled_rows_equal_matrix_rows():
    H = filt.filter_matrix(8, 6, 5, 2.5)
    for e, (idx, w) in zip([0, 17, 120, 239], filt.filter_rows(8, 6, 5, 2.5, [0, 17, 120, 239])):
        row = H.getrow(e).toarray().ravel()
        ref = np.zeros(240)
        ref[idx] = w
        np.testing.assert_allclose(row, ref, atol=0)


def test_sensitivity_filter_hand_worked_case():
    """Non-uniform field with one element below gamma, against the values worked
    by hand in tests/golden/filter_sensitivity_3x1x1.txt.  Fails if the x
    weighting, the max(gamma, x) guard or the Hs normalisation is dropped."""
    rows = np.loadtxt("tests/golden/filter_sensitivity_3x1x1.txt")
    x, dc, hs, want = rows[:, 1], rows[:, 2], rows[:, 3], rows[:, 4]
    F = filt.Filter(3, 1, 1, 1.5)
    np.testing.assert_allclose(F.Hs, hs, rtol=1e-15)
    np.testing.assert_allclose(F.sensitivity(x, dc), want, rtol=1e-14)
