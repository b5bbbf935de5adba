"""Pins of the oracle's transfer function (Eq. 4, 5-10, 25, DC reading).

Every check compares against something other than the oracle's own formula:
the independent boundary-value solve of Eq. 5-8, the limits the paper
states (Eq. 4 homogeneous; rigid base = 1 - Lambda of Eq. 25; Winkler
slope of Eq. 14-15), and a textbook closed form (Love's uniformly loaded
square) for the DC reading.
"""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle.operator import Operator
from oracle.solvers import self_influence
from oracle.transfer import (Material, bvp_surface_displacement, coeffs_ab,
                             dc_bz, brillouin_integral, khat, khat_raw,
                             shape_factor, transfer_table)

MATS = [
    Material(0.1, 10.0, 0.3, 1.0, 0.3),
    Material(0.1, 0.1, 0.3, 1.0, 0.3),
    Material(0.02, 3.0, 0.25, 1.0, 0.45),
    Material(0.5, 0.05, 0.45, 1.0, 0.2),
    Material(1.0, 100.0, 0.2, 1.0, 0.4),
]


@pytest.mark.parametrize("mat", MATS)
def test_normalised_equals_raw_eq9_10(mat):
    k = np.logspace(-3, 3, 61) / mat.h
    raw = khat_raw(k, mat)
    nrm = khat(k, mat)
    np.testing.assert_allclose(nrm, raw, rtol=1e-12, atol=0)


@pytest.mark.parametrize("mat", MATS)
@pytest.mark.parametrize("t", [1e-3, 0.05, 0.3, 1.0, 2.5, 6.0, 12.0])
def test_eq9_matches_boundary_value_problem(mat, t):
    """Eq. 9 against a direct solve of Eq. 5-8 with conditions (a)-(d)."""
    k = t / mat.h
    uz, im = bvp_surface_displacement(k, mat)
    assert im < 1e-9 * abs(uz)
    assert uz == pytest.approx(float(khat(k, mat)), rel=1e-9)


def test_bvp_homogeneous_is_eq4():
    mat = Material(0.3, 2.0, 0.35, 2.0, 0.35)
    for k in (0.1, 1.0, 10.0):
        uz, _ = bvp_surface_displacement(k, mat)
        assert uz == pytest.approx(2.0 / (mat.E1s * k), rel=1e-10)


@pytest.mark.parametrize("nu", [0.2, 0.3, 0.45])
def test_homogeneous_limit_eq4(nu):
    mat = Material(0.1, 3.0, nu, 3.0, nu)
    a, b = coeffs_ab(mat)
    assert a == 0.0 and b == 0.0
    k = np.logspace(-2, 3, 40)
    np.testing.assert_allclose(khat(k, mat), 2.0 / (mat.E1s * k), rtol=1e-15)


@pytest.mark.parametrize("mat", MATS)
def test_thin_and_thick_limits(mat):
    k = np.logspace(-1, 1, 9)
    thin = Material(1e-9, mat.E1, mat.nu1, mat.E2, mat.nu2)
    np.testing.assert_allclose(khat(k, thin), 2.0 / (mat.E2s * k), rtol=1e-7)
    thick = Material(1e3, mat.E1, mat.nu1, mat.E2, mat.nu2)
    np.testing.assert_allclose(khat(k, thick), 2.0 / (mat.E1s * k), rtol=1e-12)


@pytest.mark.parametrize("nu", [0.25, 0.3, 0.45])
def test_rigid_base_is_one_minus_lambda_eq25(nu):
    """E2 -> inf: E1* k K^ / 2 = 1 - Lambda(kh) of Eq. 25."""
    mat = Material(1.0, 1.0, nu, 1e14, 0.3)
    t = np.linspace(1e-3, 20.0, 200)
    np.testing.assert_allclose(shape_factor(t, mat), 1.0 - an.Lambda(t, nu),
                               rtol=1e-11, atol=1e-13)
    assert float(an.Lambda(1e-12, nu)) == pytest.approx(1.0, abs=1e-9)


@pytest.mark.parametrize("nu", [0.2, 0.3, 0.4])
def test_winkler_slope_eq14_15(nu):
    """Thin layer on a rigid base: K^ -> h / E~1 (Eq. 14-15)."""
    mat = Material(1.0, 2.0, nu, 1e14, 0.3)
    t = 1e-6
    slope = float(shape_factor(t, mat)) / t
    assert slope == pytest.approx(mat.E1s / (2.0 * an.e_tilde(mat.E1, nu)), rel=1e-5)
    if nu == 0.3:
        assert slope == pytest.approx(0.408163, abs=2e-6)


def test_transfer_positive_over_batch_ranges():
    rng = np.random.default_rng(11)
    worst = np.inf
    for _ in range(2000):
        mat = Material(float(np.exp(rng.uniform(np.log(1e-3), np.log(0.3)))),
                       float(np.exp(rng.uniform(np.log(0.01), np.log(100.0)))),
                       float(rng.uniform(0.2, 0.45)), 1.0,
                       float(rng.uniform(0.2, 0.45)))
        t = np.logspace(-4, 2, 60)
        worst = min(worst, float(shape_factor(t, mat).min()))
    assert worst > 0.0


def test_dc_homogeneous_closed_form():
    """Homogeneous: integral over the zone is 16 pi ln(1+sqrt2)/(E* D)."""
    mat = Material(0.0, 2.0, 0.3, 2.0, 0.3)
    N, L = 32, 2.0
    I = brillouin_integral(N, L, mat)
    assert I == pytest.approx(16 * math.pi * math.log(1 + math.sqrt(2)) / (mat.E1s * L / N), rel=1e-12)


@pytest.mark.parametrize("N", [16, 64])
def test_self_influence_is_love_square(N):
    """With the DC reading, the homogeneous self-influence of a cell equals
    the centre displacement of a uniformly loaded square of side D (Love):
    4 D ln(1 + sqrt 2) / (pi E*)."""
    mat = Material(0.0, 1.5, 0.25, 1.5, 0.25)
    L = 1.0
    op = Operator(N, L, mat)
    D = L / N
    assert self_influence(op) == pytest.approx(
        4 * D * math.log(1 + math.sqrt(2)) / (math.pi * mat.E1s), rel=1e-12)


def test_dc_limits_thin_and_thick():
    N, L = 32, 1.0
    E1, E2, nu = 4.0, 1.0, 0.3
    D = L / N
    thick = Material(1e8, E1, nu, E2, nu)
    thin = Material(1e-12, E1, nu, E2, nu)
    hom = lambda Es: 16 * math.pi * math.log(1 + math.sqrt(2)) / (Es * D)
    assert brillouin_integral(N, L, thick) == pytest.approx(hom(thick.E1s), rel=1e-8)
    assert brillouin_integral(N, L, thin) == pytest.approx(hom(thin.E2s), rel=1e-8)


def test_table_layout_and_symmetry():
    mat = MATS[0]
    N, L = 16, 1.0
    T = transfer_table(N, L, mat)
    M = 2 * N
    assert T.shape == (M, N + 1)
    # even in ky
    np.testing.assert_array_equal(T[1:], T[1:][::-1])
    # symmetric in kx <-> ky on the common quadrant
    np.testing.assert_allclose(T[: N + 1, : N + 1], T[: N + 1, : N + 1].T, rtol=1e-15)
    assert T[0, 0] == pytest.approx(dc_bz(N, L, mat), rel=1e-15)
    assert np.all(T > 0)


def test_critical_stress_eq12():
    mat = Material(0.1, 0.1, 0.3, 1.0, 0.3)
    from oracle.transfer import critical_stress
    s = critical_stress(mat, 1e-3, 2.0 / 512)
    assert s == pytest.approx(math.sqrt(0.1 / 0.91 * 1e-3 / (0.473201 * 2.0 / 512)), rel=1e-15)
    assert s == pytest.approx(0.24382, abs=1e-5)
