"""Pins of the oracle's u = K p (Eq. 1, 2, 11).

The FFT evaluation is checked against the direct O(N^4) sum of Eq. 1 with
the kernel built by explicit DFT sums, against symmetry / definiteness /
translation invariance of a convolution with an even positive kernel, and
against textbook surface displacements of the homogeneous half-space
(uniformly loaded disc, Hertz pressure).
"""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle.operator import Operator
from oracle.transfer import Material
from paper_1807_01885_amd import inputs

LAYER = Material(0.1, 10.0, 0.3, 1.0, 0.3)


@pytest.mark.parametrize("N", [4, 8, 16])
@pytest.mark.parametrize("mat", [LAYER, Material(0.02, 0.1, 0.25, 1.0, 0.45)])
def test_fft_equals_direct_sum(N, mat):
    op = Operator(N, 1.0, mat)
    rng = np.random.default_rng(N)
    p = rng.standard_normal((N, N))
    u_fft = op.apply(p)
    u_dir = op.apply_direct(p)
    np.testing.assert_allclose(u_fft, u_dir, rtol=0, atol=1e-12 * np.abs(u_dir).max())
    _, imag = op.kernel_direct()
    assert imag < 1e-12


def test_symmetric_positive_definite():
    op = Operator(32, 1.0, LAYER)
    rng = np.random.default_rng(1)
    p = rng.standard_normal((32, 32))
    q = rng.standard_normal((32, 32))
    a = np.sum(op.apply(p) * q)
    b = np.sum(p * op.apply(q))
    assert a == pytest.approx(b, rel=1e-12)
    for _ in range(5):
        x = rng.standard_normal((32, 32))
        assert np.sum(x * op.apply(x)) > 0


def test_translation_invariance():
    N = 32
    op = Operator(N, 1.0, LAYER)
    p = np.zeros((N, N))
    p[10:14, 9:12] = 1.0
    q = np.roll(np.roll(p, 3, axis=0), -2, axis=1)
    up = op.apply(p)
    uq = op.apply(q)
    np.testing.assert_allclose(np.roll(np.roll(up, 3, axis=0), -2, axis=1)[8:24, 8:24],
                               uq[8:24, 8:24], rtol=1e-12)


def test_batch_apply_matches_single():
    op = Operator(16, 1.0, LAYER)
    rng = np.random.default_rng(2)
    ps = rng.standard_normal((3, 16, 16))
    ub = op.apply_batch(ps)
    for i in range(3):
        np.testing.assert_allclose(ub[i], op.apply(ps[i]), rtol=1e-13, atol=1e-16)


def test_uniform_disc_displacement():
    """Homogeneous: uniform p0 on a disc, u(0) = 2 p0 a/E*, u(a) = 4 p0 a/(pi E*)."""
    N, L = 512, 1.0
    mat = Material(0.0, 1.0, 0.3, 1.0, 0.3)
    op = Operator(N, L, mat)
    X, Y = inputs.coords(N, L)
    a = L / 8
    p = (X * X + Y * Y <= a * a).astype(float)
    u = op.apply(p)
    u0, ua = an.uniform_disc_displacement(1.0, a, mat.E1s)
    c = N // 2
    assert u[c, c] == pytest.approx(u0, rel=3e-3)
    # edge: average of the four axis points straddling r = a
    j = c + int(round(a / (L / N)))
    edge = 0.5 * (u[c, j - 1] + u[c, j])
    assert edge == pytest.approx(ua, rel=2e-2)


def test_hertz_pressure_displacement():
    """Homogeneous: Hertz pressure gives u = pi p0 (2a^2 - r^2)/(4 a E*)."""
    N, L = 256, 1.0
    mat = Material(0.0, 1.0, 0.3, 1.0, 0.3)
    op = Operator(N, L, mat)
    X, Y = inputs.coords(N, L)
    r = np.sqrt(X * X + Y * Y)
    a, p0 = L / 8, 1.0
    u = op.apply(an.hertz_pressure(r, a, p0))
    inside = r < 0.8 * a
    ref = an.hertz_pressure_displacement(r[inside], a, p0, mat.E1s)
    np.testing.assert_allclose(u[inside], ref, rtol=3e-3)
