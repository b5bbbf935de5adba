"""Pins of the multi-layer transfer function (the boundary-value problem of
Eq. 5-8 written for a stack of bonded layers) and the library's host table
for layered plans against it.

Oracle pins: one layer is Eq. 9 (closed form, independently typed); no
layer is Eq. 4; splitting a layer into identical sublayers, or adding a
bottom layer of the half-space's own material, changes nothing; the limits
k -> inf (top layer) and k -> 0 (half-space); and the Brillouin-zone
integral of one layer equals the single-layer oracle's.
"""
import ctypes
import math
import os

import numpy as np
import pytest

from oracle.multilayer import (brillouin_integral_layers, khat_layers, surface_compliance,
                               transfer_table_layers)
from oracle.transfer import Material, brillouin_integral, khat, transfer_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1807_01885_amd", "libcoatbem.so")

STACKS = [
    ([(0.02, 10.0, 0.3), (0.05, 0.5, 0.45)], 1.0, 0.25),
    ([(0.01, 0.1, 0.2), (0.03, 30.0, 0.35), (0.2, 2.0, 0.3)], 1.0, 0.3),
    ([(0.005, 100.0, 0.25), (0.001, 0.01, 0.4)], 3.0, 0.2),
]


@pytest.mark.parametrize("mat", [Material(0.1, 10.0, 0.3, 1.0, 0.25), Material(0.02, 0.05, 0.45, 1.0, 0.2),
                                 Material(1.0, 1.0, 0.3, 1e5, 0.3)])
def test_one_layer_is_eq9(mat):
    for kh in np.logspace(-3, 2.3, 23):
        k = kh / mat.h
        a = surface_compliance(k, [(mat.h, mat.E1, mat.nu1)], mat.E2, mat.nu2)
        assert a == pytest.approx(float(khat(k, mat)), rel=1e-12)


def test_no_layer_is_eq4():
    for k in (1e-2, 1.0, 300.0):
        assert surface_compliance(k, [], 2.0, 0.35) == pytest.approx(2.0 * (1 - 0.35 ** 2) / (2.0 * k), rel=1e-13)


@pytest.mark.parametrize("layers,Es,nus", STACKS)
def test_stack_identities_and_limits(layers, Es, nus):
    H = sum(h for h, _, _ in layers)
    for k in (0.1 / H, 1.0 / H, 5.0 / H, 40.0 / layers[0][0]):
        base = surface_compliance(k, layers, Es, nus)
        assert base > 0
        # split the top layer into two identical halves
        h0, E0, n0 = layers[0]
        split = [(h0 / 3, E0, n0), (2 * h0 / 3, E0, n0)] + layers[1:]
        assert surface_compliance(k, split, Es, nus) == pytest.approx(base, rel=1e-12)
        # a bottom layer of the half-space's own material is no layer
        assert surface_compliance(k, layers + [(0.7 * H, Es, nus)], Es, nus) == pytest.approx(base, rel=1e-12)
    E1s = layers[0][1] / (1 - layers[0][2] ** 2)
    Ess = Es / (1 - nus ** 2)
    k = 200.0 / layers[0][0]
    assert surface_compliance(k, layers, Es, nus) * E1s * k / 2 == pytest.approx(1.0, rel=1e-10)
    k = 1e-7 / H
    assert surface_compliance(k, layers, Es, nus) * Ess * k / 2 == pytest.approx(1.0, rel=1e-5)


def test_brillouin_integral_one_layer():
    mat = Material(0.05, 10.0, 0.3, 1.0, 0.25)
    a = brillouin_integral_layers(64, 2.0, [(mat.h, mat.E1, mat.nu1)], mat.E2, mat.nu2)
    assert a == pytest.approx(brillouin_integral(64, 2.0, mat), rel=1e-10)


@pytest.fixture(scope="module")
def clib():
    if not os.path.exists(LIB):
        from paper_1807_01885_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def _host_table(clib, N, L, layers, Es, nus):
    f = clib.cb_transfer_table_layered
    D = ctypes.c_double
    f.argtypes = [ctypes.c_int, D, ctypes.c_int] + [ctypes.POINTER(D)] * 3 + [D, D, ctypes.c_int,
                                                                              ctypes.POINTER(D), ctypes.POINTER(D)]
    n = len(layers)
    arr = lambda q: (D * n)(*[l[q] for l in layers])
    out = np.zeros((N + 1, N + 1))
    k00 = D()
    rc = f(N, L, n, arr(0), arr(1), arr(2), Es, nus, 0, out.ctypes.data_as(ctypes.POINTER(D)), ctypes.byref(k00))
    return rc, out, k00.value


@pytest.mark.parametrize("N,L", [(16, 1.0), (64, 2.0)])
@pytest.mark.parametrize("layers,Es,nus", STACKS)
def test_host_layered_table_matches_oracle(clib, N, L, layers, Es, nus):
    rc, out, _ = _host_table(clib, N, L, layers, Es, nus)
    assert rc == 0
    ref = transfer_table_layers(N, L, layers, Es, nus)[: N + 1, : N + 1]
    np.testing.assert_allclose(out[1:, :], ref[1:, :], rtol=1e-11, atol=0)
    np.testing.assert_allclose(out[0, 1:], ref[0, 1:], rtol=1e-11, atol=0)
    # the DC value carries the Brillouin-zone quadrature of both sides
    assert out[0, 0] == pytest.approx(ref[0, 0], rel=1e-10)


def test_host_layered_table_one_layer_equals_closed_form(clib):
    mat = Material(0.1, 10.0, 0.3, 1.0, 0.25)
    N, L = 64, 4.0
    rc, out, _ = _host_table(clib, N, L, [(mat.h, mat.E1, mat.nu1)], mat.E2, mat.nu2)
    assert rc == 0
    ref = transfer_table(N, L, mat)[: N + 1, : N + 1]
    np.testing.assert_allclose(out, ref, rtol=1e-11, atol=0)


def test_host_layered_rejects_bad_stacks(clib):
    for layers in ([], [(0.0, 1.0, 0.3)], [(0.1, 1.0, 0.5)], [(0.1, -1.0, 0.3)], [(0.1, 1.0, 0.3)] * 9):
        rc, _, _ = _host_table(clib, 32, 1.0, layers, 1.0, 0.3)
        assert rc == -1
