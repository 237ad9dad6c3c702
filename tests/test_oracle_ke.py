"""Pins of the oracle's H8 element stiffness (Finite Element Analysis section).

Each check is independent of the oracle's B^T D B construction: closed forms of
linear elasticity, an exact tensor-form integration written here, rigid-body
kinematics and quadrature exactness.
"""

import itertools
import math

import numpy as np
import pytest

from oracle.ke import CORNERS, element_stiffness, rigid_body_modes


def lame(nu, E=1.0):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def tensor_form_ke(nu):
    """K^{ij}_{ab} = int lam d_i N_a d_j N_b + mu (d_j N_a d_i N_b + delta_ij grad N_a . grad N_b),
    integrated exactly with the 1D moments of (1-t), t and their derivatives."""
    lam, mu = lame(nu)
    # 1D factor of corner coordinate s in {0, 1}: value t (s=1) or 1-t (s=0), slope +-1
    def m_vv(s, r):  # int f_s f_r dt
        return 1.0 / 3.0 if s == r else 1.0 / 6.0

    def m_dv(s, r):  # int f_s' f_r dt
        return (1.0 if s == 1 else -1.0) * 0.5

    def m_dd(s, r):  # int f_s' f_r' dt
        return (1.0 if s == 1 else -1.0) * (1.0 if r == 1 else -1.0)

    def g(a, b, p, q):  # int d_p N_a d_q N_b over the unit cube
        val = 1.0
        for d in range(3):
            s, r = int(CORNERS[a, d]), int(CORNERS[b, d])
            if d == p and d == q:
                val *= m_dd(s, r)
            elif d == p:
                val *= m_dv(s, r)
            elif d == q:
                val *= m_dv(r, s)
            else:
                val *= m_vv(s, r)
        return val

    K = np.zeros((24, 24))
    for a, b in itertools.product(range(8), range(8)):
        lap = sum(g(a, b, k, k) for k in range(3))
        for i, j in itertools.product(range(3), range(3)):
            K[3 * a + i, 3 * b + j] = lam * g(a, b, i, j) + mu * (g(a, b, j, i) + (lap if i == j else 0.0))
    return K


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_ke_equals_exact_tensor_form(nu):
    np.testing.assert_allclose(element_stiffness(nu), tensor_form_ke(nu), atol=1e-14, rtol=0)


def test_ke_symmetric_and_rank():
    KE = element_stiffness(0.3)
    assert np.abs(KE - KE.T).max() < 1e-15
    ev = np.linalg.eigvalsh(KE)
    assert np.sum(np.abs(ev) < 1e-12) == 6
    assert np.sum(ev > 1e-6) == 18


def test_ke_rigid_body_null_space():
    KE = element_stiffness(0.3)
    R = rigid_body_modes()
    assert np.linalg.matrix_rank(R) == 6
    assert np.abs(KE @ R).max() < 1e-14


def test_ke_diagonal_closed_form():
    # K_00 = int (lam+2mu) N_x^2 + mu (N_y^2 + N_z^2) with N = (1-x)(1-y)(1-z): each
    # squared derivative integrates to 1/9, so K_00 = (lam + 4 mu)/9 (0.235043 at nu=0.3).
    lam, mu = lame(0.3)
    KE = element_stiffness(0.3)
    np.testing.assert_allclose(np.diag(KE), (lam + 4 * mu) / 9.0, rtol=1e-14)
    assert abs(KE[0, 0] - 0.235043) < 1e-6


def test_ke_quadrature_exact_at_two_points():
    np.testing.assert_allclose(element_stiffness(0.3, order=2), element_stiffness(0.3, order=4),
                               atol=1e-15)


@pytest.mark.parametrize("which", range(6))
def test_ke_constant_strain_energy(which):
    # nodal values of the linear field u = eps . x give a uniform strain; the strain
    # energy 2W = lam (tr eps)^2 + 2 mu eps:eps over the unit volume.
    lam, mu = lame(0.3)
    eps = np.zeros((3, 3))
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    i, j = pairs[which]
    eps[i, j] = eps[j, i] = 0.7 if i != j else 1.3
    u = np.concatenate([eps @ CORNERS[a] for a in range(8)])
    KE = element_stiffness(0.3)
    expected = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
    assert abs(u @ KE @ u - expected) < 1e-13


def test_ke_bending_mode_energy():
    # u_x = (x - 1/2)(y - 1/2): eps_xx = y - 1/2, gamma_xy = x - 1/2, so
    # 2W = int (lam + 2mu)(y-1/2)^2 + mu (x-1/2)^2 = (lam + 3 mu)/12.
    lam, mu = lame(0.3)
    u = np.zeros(24)
    for a in range(8):
        x, y, _ = CORNERS[a]
        u[3 * a] = (x - 0.5) * (y - 0.5)
    assert abs(u @ element_stiffness(0.3) @ u - (lam + 3 * mu) / 12.0) < 1e-14


def test_ke_cube_symmetry():
    # mirror x -> 1 - x maps corner a to its partner and flips the x component
    KE = element_stiffness(0.3)
    perm = []
    for a in range(8):
        x, y, z = CORNERS[a]
        perm.append(int(np.nonzero((CORNERS == [1 - x, y, z]).all(axis=1))[0][0]))
    T = np.zeros((24, 24))
    for a in range(8):
        for c in range(3):
            T[3 * perm[a] + c, 3 * a + c] = -1.0 if c == 0 else 1.0
    np.testing.assert_allclose(T @ KE @ T.T, KE, atol=1e-15)
    assert math.isclose(np.linalg.eigvalsh(KE).max(), np.linalg.eigvalsh(T @ KE @ T.T).max())
