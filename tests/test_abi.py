"""CPU checks of the C-ABI library: it loads, exports every symbol the
header declares, rejects bad arguments, and its host-side transfer table
(Eq. 9-11 with the DC rule) agrees with the oracle.  No device compute."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.operator import Operator
from oracle.solvers import self_influence
from oracle.transfer import Material, transfer_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1807_01885_amd", "libcoatbem.so")
HEADER = os.path.join(ROOT, "include", "coatbem.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1807_01885_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cb_[a-z_A-Z0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), f"{n} declared in coatbem.h but not exported"


def test_binding_covers_header():
    src = open(os.path.join(ROOT, "paper_1807_01885_amd", "coatbem.py")).read()
    for n in declared_functions():
        assert f'"{n}"' in src, f"binding lacks {n}"


def _table(lib, N, L, m, dc_mode=0):
    f = lib.cb_transfer_table
    f.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6 + [
        ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    out = np.zeros((N + 1, N + 1))
    k00 = ctypes.c_double()
    rc = f(N, L, m.h, m.E1, m.nu1, m.E2, m.nu2, dc_mode,
           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(k00))
    return rc, out, k00.value


@pytest.mark.parametrize("N,L,m", [
    (64, 4.0, Material(0.1, 10.0, 0.3, 1.0, 0.3)),
    (512, 2.0, Material(0.02, 0.1, 0.3, 1.0, 0.3)),
    (256, 1.0, Material(0.0, 1.0, 0.3, 1.0, 0.3)),
    (128, 1.0, Material(0.5, 0.05, 0.45, 1.0, 0.2)),
    (32, 1.0, Material(1e-3, 100.0, 0.2, 1.0, 0.45)),
])
def test_host_table_matches_oracle(lib, N, L, m):
    rc, out, k00 = _table(lib, N, L, m)
    assert rc == 0
    ref = transfer_table(N, L, m)[: N + 1, : N + 1]
    np.testing.assert_allclose(out, ref, rtol=1e-11, atol=0)
    assert k00 == pytest.approx(self_influence(Operator(N, L, m)), rel=1e-12)


@pytest.mark.parametrize("idx", [1, 4, 5, 65, 87])
def test_host_table_dc_stiff_coatings(lib, idx):
    """The Brillouin-zone DC value on the recipe's stiffest coatings (E1/E2 up
    to 88, h/L down to 1e-3), where C(kh) has a narrow peak of height about
    E1*/E2* at k = 0: library quadrature against the oracle's adaptive one."""
    from paper_1807_01885_amd import inputs
    from oracle.transfer import dc_bz
    c = (inputs.batch_c4(n=64, seed=4) + inputs.headline_set())[idx]
    N = min(c.N, 256)
    m = Material(c.h, c.E1, c.nu1, c.E2, c.nu2)
    rc, out, _ = _table(lib, N, c.L, m)
    assert rc == 0
    assert out[0, 0] == pytest.approx(dc_bz(N, c.L, m), rel=1e-12)


def test_host_table_dc_zero(lib):
    m = Material(0.1, 10.0, 0.3, 1.0, 0.3)
    rc, out, _ = _table(lib, 32, 1.0, m, dc_mode=1)
    assert rc == 0 and out[0, 0] == 0.0


@pytest.mark.parametrize("args", [
    (15, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3),      # N not a power of two
    (8192, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3),    # N too large
    (64, 0.0, 0.1, 1.0, 0.3, 1.0, 0.3),      # L = 0
    (64, 1.0, -0.1, 1.0, 0.3, 1.0, 0.3),     # h < 0
    (64, 1.0, 0.1, -1.0, 0.3, 1.0, 0.3),     # E1 < 0
    (64, 1.0, 0.1, 1.0, 0.5, 1.0, 0.3),      # nu = 0.5
    (64, 1.0, 0.1, 1.0, 0.3, float("nan"), 0.3),
])
def test_invalid_parameters_rejected(lib, args):
    m = Material(args[2], args[3], args[4], args[5], args[6])
    rc, _, _ = _table(lib, args[0], args[1], m)
    assert rc == -1
    lib.cb_last_error.restype = ctypes.c_char_p
    assert len(lib.cb_last_error()) > 0


def test_plan_create_rejects_before_touching_device(lib):
    f = lib.cb_plan_create
    f.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int] + [ctypes.c_double] * 7 + [ctypes.c_void_p]
    h = ctypes.c_void_p(1)
    assert f(ctypes.byref(h), 100, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3, 0.0, None) == -1
    assert h.value is None
    assert f(None, 64, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3, 0.0, None) == -1


def test_null_plan_calls_are_errors(lib):
    lib.cb_apply_K.argtypes = [ctypes.c_void_p] * 3
    assert lib.cb_apply_K(None, None, None) == -1
    assert lib.cb_plan_destroy(None) == 0
    lib.cb_status_string.restype = ctypes.c_char_p
    assert lib.cb_status_string(-4) == b"not converged"
    assert lib.cb_version() >= 100
