"""Pins of the literal periodic operator (Eq. 11 without padding, no DC
component) and of force-controlled contact on it.

  * Eq. 3-4 / Eq. 9: a harmonic load p0 cos(k.x) with k a grid wavenumber
    is an eigenfunction; u = K^(|k|) p0 cos(k.x) exactly, from the closed
    form, not from the FFT table.
  * The sum of Eq. 11 written out with explicit exponentials (O(N^4)).
  * No DC component: a uniform pressure gives u = 0, every u has zero mean.
  * Force control on it against a brute-force QP (NNLS on K + c 1 1^T).
  * Westergaard's wavy contact on the homogeneous half-space (Johnson,
    Contact Mechanics, Sec. 13.2): full contact at p_mean >= p* with
    p = p_mean + p* cos(2 pi x / lambda), p* = pi E* g0 / lambda, exactly on
    the grid; partial contact of half-width a = (lambda/pi) asin(sqrt(p_mean/p*)).
"""
import math

import numpy as np
import pytest

from oracle.periodic import PeriodicOperator
from oracle.solvers import solve_nnls_force_singular, solve_pk
from oracle.transfer import Material, khat
from paper_1807_01885_amd import inputs

LAYER = Material(0.05, 10.0, 0.3, 1.0, 0.25)
SOFT = Material(0.02, 0.1, 0.45, 1.0, 0.3)


@pytest.mark.parametrize("mat", [LAYER, SOFT])
def test_harmonic_load_is_an_eigenfunction(mat):
    N, L = 64, 2.0
    op = PeriodicOperator(N, L, mat)
    X, Y = inputs.coords(N, L)
    for (a, b) in ((1, 0), (3, 5), (0, 31), (17, 9), (32, 32)):
        kx, ky = 2 * np.pi * a / L, 2 * np.pi * b / L
        p = np.cos(kx * X + ky * Y + 0.3)
        u = op.apply(p)
        ref = float(khat(math.hypot(kx, ky), mat)) * p
        assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def test_direct_sum_and_no_dc():
    N, L = 12, 1.0
    op = PeriodicOperator(N, L, LAYER)
    rng = np.random.default_rng(3)
    p = rng.standard_normal((N, N))
    u = op.apply(p)
    ud = op.apply_direct(p)
    assert np.abs(u - ud).max() <= 1e-12 * np.abs(ud).max()
    assert abs(u.mean()) <= 1e-14 * np.abs(u).max()
    assert np.abs(op.apply(np.full((N, N), 7.0))).max() <= 1e-14


@pytest.mark.parametrize("shape", ["paraboloid", "rough"])
def test_periodic_force_control_equals_brute_force(shape):
    N, L = 10, 1.0
    op = PeriodicOperator(N, L, LAYER)
    f = inputs.paraboloid(N, L, 1.0) if shape == "paraboloid" else inputs.rough_surface(N, L, seed=2)
    F = 2e-3 if shape == "paraboloid" else 1e-4
    r = solve_pk(op, f, F, mode="force", tol=1e-12)
    assert r.converged and r.F == pytest.approx(F, rel=1e-12)
    pn, dn = solve_nnls_force_singular(op, f, F)
    assert 0 < (pn > 0).sum() < N * N
    assert np.array_equal(r.p > 0, pn > 0)
    np.testing.assert_allclose(r.p, pn, rtol=0, atol=1e-8 * pn.max())
    assert r.d == pytest.approx(dn, rel=1e-8, abs=1e-12 * L)


def test_westergaard_full_contact_exact():
    N, L, g0 = 64, 1.0, 1e-3
    mat = Material(0.0, 2.0, 0.3, 2.0, 0.3)
    op = PeriodicOperator(N, L, mat)
    X, _ = inputs.coords(N, L)
    f = g0 * (1.0 - np.cos(2 * np.pi * X / L))
    pstar = math.pi * mat.E1s * g0 / L
    pbar = 1.5 * pstar
    r = solve_pk(op, f, pbar * L * L, mode="force", tol=1e-12)
    ref = pbar + pstar * np.cos(2 * np.pi * X / L)
    assert r.converged
    assert np.abs(r.p - ref).max() <= 1e-9 * pstar
    assert r.d == pytest.approx(g0, rel=1e-9)


@pytest.mark.parametrize("ratio", [0.25, 0.6])
def test_westergaard_partial_contact(ratio):
    N, L, g0 = 256, 1.0, 1e-3
    mat = Material(0.0, 2.0, 0.3, 2.0, 0.3)
    op = PeriodicOperator(N, L, mat)
    X, _ = inputs.coords(N, L)
    f = g0 * (1.0 - np.cos(2 * np.pi * X / L))
    pstar = math.pi * mat.E1s * g0 / L
    pbar = ratio * pstar
    r = solve_pk(op, f, pbar * L * L, mode="force", tol=1e-11)
    assert r.converged
    a = L / math.pi * math.asin(math.sqrt(ratio))
    width = (r.p[N // 2] > 0).sum() * op.dx
    assert width == pytest.approx(2 * a, abs=2.5 * op.dx)
    # every row carries the same 1-D solution
    assert np.abs(r.p - r.p[N // 2][None, :]).max() <= 1e-8 * r.p.max()
