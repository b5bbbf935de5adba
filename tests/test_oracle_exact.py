"""Exact influence coefficients of uniformly loaded square cells (Eq. 1 with
piecewise-constant pressure, the inverse transform of Eq. 9-11): the oracle
(oracle/exact.py) pinned by closed forms, limits and a real-space brute force,
and the library's host-side coefficients and table (cb_transfer_table_exact)
against it.  CPU only."""
import ctypes
import math
import os

import numpy as np
import pytest
import scipy.integrate as si

from oracle.exact import (Coating, ExactOperator, Stack, exact_table, influence_grid, influence_points, love_rect,
                          remainder_points, softened_rect)
from oracle.transfer import Material, shape_factor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1807_01885_amd", "libcoatbem.so")
_d = ctypes.c_double
_pd = ctypes.POINTER(_d)


# ---------------------------------------------------------------------------
# oracle pins
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("x,y", [(0.3, 0.1), (0.05, 0.0), (1.0, 0.7)])
def test_love_against_brute_force(x, y):
    """Love's rectangle formula against dblquad of 1/(pi E* r) over the
    rectangle (points outside it)."""
    a, b, Es = 0.02, 0.03, 1.7
    ref, _ = si.dblquad(lambda yy, xx: 1.0 / (math.pi * Es * math.hypot(x - xx, y - yy)), -a, a, -b, b,
                        epsabs=0, epsrel=1e-13)
    assert float(love_rect(x, y, a, b, Es)) == pytest.approx(ref, rel=1e-11)


def test_love_centre_of_square():
    """Centre of a uniformly loaded square of side 2a: in polar form
    (8/(pi E*)) int_0^{pi/4} a/cos(t) dt = (8 a/(pi E*)) ln(1 + sqrt 2)."""
    a, Es = 0.25, 2.0
    assert float(love_rect(0.0, 0.0, a, a, Es)) == pytest.approx(8 * a * math.log(1 + math.sqrt(2)) / (math.pi * Es),
                                                                 rel=1e-15)


@pytest.mark.parametrize("x,y", [(0.0, 0.0), (0.07, 0.0), (0.2, 0.15)])
def test_softened_rect_against_brute_force(x, y):
    a, beta = 0.03, 0.05
    ref, _ = si.dblquad(lambda yy, xx: 1.0 / math.sqrt((x - xx) ** 2 + (y - yy) ** 2 + beta ** 2), -a, a, -a, a,
                        epsabs=0, epsrel=1e-13)
    assert float(softened_rect(x, y, a, a, beta)) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("x,y", [(0.0, 0.0), (1 / 32, 0.0), (0.1, 0.03), (0.5, 0.4)])
def test_fourier_polar_against_closed_form(x, y):
    """psi(k) = c e^{-b k} is the transform of c / (2 pi sqrt(r^2 + b^2)):
    the polar Fourier integral over the cell must equal (c / 2 pi) times
    the closed rectangle integral (tests the cell transform, the 1/4 pi^2,
    the t-trapezoid and the k-rule together)."""
    a, c, b = 1 / 64, 0.7, 0.05
    v = remainder_points([x], [y], a, lambda k: c * np.exp(-b * k), 40 / b, 0.25 / b, 0.01 / b)[0]
    assert v == pytest.approx(c / (2 * math.pi) * float(softened_rect(x, y, a, a, b)), rel=1e-12)


def _g_brute(r, mat):
    """(1/2 pi) int_0^inf psi(k) J0(k r) dk, psi = (2/E1*)(C(kh) - 1), with
    J0(z) = (2/pi) int_0^{pi/2} cos(z cos phi) dphi: inner Fourier cosine
    integrals by QUADPACK's QAWF, outer by quad."""
    psi = lambda k: (2 / mat.E1s) * (float(shape_factor(k * mat.h, mat)) - 1.0)

    def inner(phi):
        return si.quad(psi, 0, np.inf, weight="cos", wvar=r * math.cos(phi), limlst=200)[0]

    return si.quad(inner, 0, math.pi / 2, epsabs=0, epsrel=1e-12, limit=200)[0] / math.pi ** 2


@pytest.mark.parametrize("mat", [Material(0.1, 10.0, 0.3, 1.0, 0.3), Material(0.05, 0.1, 0.3, 1.0, 0.25)])
def test_coated_coefficient_against_real_space_brute_force(mat):
    """The coated part of a cell coefficient at offset (3, 1) cells: the
    Fourier-polar integral against the cell integral (8 x 8 Gauss-Legendre,
    the integrand is smooth there) of the point-load Green's function
    computed by a different route (cosine transforms)."""
    dx = 1 / 32
    a, x, y = dx / 2, 3 * dx, dx
    g, w = np.polynomial.legendre.leggauss(8)
    ref = a * a * sum(w[i] * w[j] * _g_brute(math.hypot(x + a * g[i], y + a * g[j]), mat)
                      for i in range(8) for j in range(8))
    b = Coating(mat)
    assert remainder_points([x], [y], a, b.psi, b.kmax, b.kscale, b.kfirst)[0] == pytest.approx(ref, rel=1e-11)


def test_homogeneous_and_limits():
    """E1 = E2 (any h): Love's coefficients of that modulus.  A coating much
    thicker than the patch: the coating's own half-space, the departure
    falling like 1/h.  A coating much thinner than the cell: the
    substrate's, the departure shrinking with h."""
    N, dx = 8, 1 / 8
    pos = np.arange(N + 1) * dx
    X, Y = np.meshgrid(pos, pos, indexing="ij")
    m = Material(0.1, 2.0, 0.3, 2.0, 0.3)
    D = influence_grid(N, dx, Coating(m))
    np.testing.assert_allclose(D, love_rect(X, Y, dx / 2, dx / 2, m.E1s), rtol=1e-13)
    dev = []
    for h in (100.0, 1000.0):
        thick = Material(h, 3.0, 0.3, 1.0, 0.3)
        D = influence_grid(N, dx, Coating(thick))
        dev.append(np.max(np.abs(D / love_rect(X, Y, dx / 2, dx / 2, thick.E1s) - 1)))
    assert dev[1] < 3.5e-3 and dev[0] / dev[1] == pytest.approx(10.0, rel=0.02)
    ms, qs = np.array([0, 1, 2]), np.array([0, 0, 1])
    dev = []
    for h in (dx / 10, dx / 40):
        thin = Material(h, 3.0, 0.3, 1.0, 0.3)
        D = influence_points(ms, qs, dx, Coating(thin))
        dev.append(np.abs(D / love_rect(ms * dx, qs * dx, dx / 2, dx / 2, thin.E2s) - 1))
    assert np.all(dev[1] < dev[0]) and np.all(dev[1] < [0.03, 2e-3, 5e-4])


@pytest.mark.parametrize("mat", [Material(0.1, 10.0, 0.3, 1.0, 0.3), Material(0.05, 0.1, 0.3, 1.0, 0.25)])
def test_additivity_of_cells(mat):
    """A 3 x 3 block of cells of side Delta is one cell of side 3 Delta: the
    sum of nine coefficients equals the big cell's coefficient."""
    dx = 1 / 64
    pts = [(10, 4), (3, 3), (0, 0)]
    small = influence_points([m + i for (m, q) in pts for i in (-1, 0, 1) for j in (-1, 0, 1)],
                             [q + j for (m, q) in pts for i in (-1, 0, 1) for j in (-1, 0, 1)], dx, Coating(mat))
    big = influence_points([m / 3 for (m, q) in pts], [q / 3 for (m, q) in pts], 3 * dx, Coating(mat))
    np.testing.assert_allclose(small.reshape(3, 9).sum(axis=1), big, rtol=1e-11)


def test_fft_apply_equals_direct_sum():
    """The DC-FFT table reproduces u_i = sum_j D[|i-j|] p_j exactly."""
    op = ExactOperator(16, 1.0, Material(0.1, 10.0, 0.3, 1.0, 0.3))
    p = np.random.default_rng(0).random((16, 16))
    np.testing.assert_allclose(op.apply(p), op.apply_direct(p), rtol=1e-12, atol=0)


def test_exact_operator_loaded_square_is_love():
    """Homogeneous half-space, uniform pressure on a K x K block of cells: the
    displacement at every cell centre is Love's formula for the block."""
    N, dx, Es = 32, 1 / 32, 1.0 / 0.91
    op = ExactOperator(N, 1.0, Material(0.1, 1.0, 0.3, 1.0, 0.3))
    p = np.zeros((N, N))
    p[8:16, 4:16] = 1.0
    u = op.apply(p)
    c = (np.arange(N) + 0.5) * dx
    X, Y = np.meshgrid(c, c, indexing="ij")
    ref = love_rect(X - 12 * dx, Y - 10 * dx, 4 * dx, 6 * dx, Es)
    np.testing.assert_allclose(u, ref, rtol=1e-12)


# ---------------------------------------------------------------------------
# library host-side coefficients against the oracle
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def clib():
    if not os.path.exists(LIB):
        from paper_1807_01885_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(LIB)
    lib.cb_transfer_table_exact.argtypes = [ctypes.c_int] + [_d] * 6 + [_pd, _pd]
    lib.cb_transfer_table_exact_layered.argtypes = [ctypes.c_int, _d, ctypes.c_int, _pd, _pd, _pd, _d, _d, _pd, _pd]
    return lib


def _lib_exact(lib, N, L, m):
    T = np.zeros((N + 1, N + 1))
    D = np.zeros((N + 1, N + 1))
    rc = lib.cb_transfer_table_exact(N, L, m.h, m.E1, m.nu1, m.E2, m.nu2, T.ctypes.data_as(_pd), D.ctypes.data_as(_pd))
    return rc, T, D


@pytest.mark.parametrize("N,m", [
    (16, Material(0.1, 10.0, 0.3, 1.0, 0.3)),
    (32, Material(0.05, 0.1, 0.3, 1.0, 0.25)),
    (64, Material(0.2, 3.0, 0.35, 1.0, 0.2)),
    (16, Material(1 / 64, 5.0, 0.3, 1.0, 0.3)),       # h = Delta / 4
    (32, Material(0.1, 100.0, 0.3, 1.0, 0.3)),        # stiff: C has a pole next to k = 0
    (16, Material(0.05, 1.0, 0.2, 1.0, 0.4)),         # equal E, different nu
])
def test_library_coefficients_full_grid(clib, N, m):
    rc, T, D = _lib_exact(clib, N, 1.0, m)
    assert rc == 0
    Do = influence_grid(N, 1.0 / N, Coating(m))
    np.testing.assert_allclose(D, Do, rtol=1e-12, atol=0)
    To = exact_table(Do)[: N + 1, :]
    assert np.max(np.abs(T - To)) <= 1e-13 * np.max(np.abs(To))


def _sample(N, rng, n=16):
    ms = np.concatenate([[0, 1, 2, 3, N, N, 5, N // 2], rng.integers(0, N + 1, n)])
    qs = np.concatenate([[0, 0, 1, 3, N, 0, 2, N // 3], rng.integers(0, N + 1, n)])
    return ms, qs


@pytest.mark.parametrize("N,m,near,rtol", [
    (1024, Material(0.05, 10.0, 0.3, 1.0, 0.3), False, 1e-12),
    (1024, Material(1.0001 / 8192, 0.5, 0.3, 1.0, 0.3), True, 1e-12),   # the thinnest top layer accepted
    (1024, Material(0.02, 1e4, 0.3, 1.0, 0.3), False, 1e-11),
    (512, Material(0.3, 0.01, 0.45, 1.0, 0.2), False, 1e-10),  # far field = a 1% difference of the two parts
])
def test_library_coefficients_sampled(clib, N, m, near, rtol):
    """Full-size grids: sampled offsets (near the origin, at the far corner,
    random), the oracle one offset set at a time (for the thinnest layer
    only offsets near the origin: its k range makes far ones too costly)."""
    rc, T, D = _lib_exact(clib, N, 1.0, m)
    assert rc == 0
    rng = np.random.default_rng(N)
    ms, qs = (np.array([0, 1, 2, 3, 5, 6]), np.array([0, 0, 1, 3, 2, 6])) if near else _sample(N, rng)
    Do = influence_points(ms, qs, 1.0 / N, Coating(m))
    np.testing.assert_allclose(D[ms, qs], Do, rtol=rtol, atol=0)
    np.testing.assert_array_equal(D, D.T)


def test_library_layered_coefficients(clib):
    layers = [(0.02, 5.0, 0.3), (0.05, 0.5, 0.25)]
    N = 128
    T = np.zeros((N + 1, N + 1))
    D = np.zeros((N + 1, N + 1))
    arr = lambda k: (_d * 2)(*[l[k] for l in layers])
    rc = clib.cb_transfer_table_exact_layered(N, 1.0, 2, arr(0), arr(1), arr(2), 1.0, 0.3, T.ctypes.data_as(_pd),
                                              D.ctypes.data_as(_pd))
    assert rc == 0
    ms, qs = _sample(N, np.random.default_rng(1))
    np.testing.assert_allclose(D[ms, qs], influence_points(ms, qs, 1.0 / N, Stack(layers, 1.0, 0.3)), rtol=1e-12)


def test_library_half_space_and_thin_limit(clib):
    """h = 0 is the substrate alone (Love's coefficients of E2*); a top layer
    thinner than Delta/8 is refused (CB_E_UNSUPPORTED = -7)."""
    N = 64
    rc, T, D = _lib_exact(clib, N, 1.0, Material(0.0, 2.0, 0.3, 1.0, 0.25))
    assert rc == 0
    pos = np.arange(N + 1) / N
    X, Y = np.meshgrid(pos, pos, indexing="ij")
    np.testing.assert_allclose(D, love_rect(X, Y, 0.5 / N, 0.5 / N, 1.0 / (1 - 0.25 ** 2)), rtol=1e-13)
    rc, _, _ = _lib_exact(clib, N, 1.0, Material(1.0 / (9 * N), 2.0, 0.3, 1.0, 0.25))
    assert rc == -7
