"""GPU parity of cb_apply_precond, the solver's Fourier preconditioners
(the N-periodic convolution: the same three kernels as cb_apply_K without
the zero padding), against numpy's periodic real FFT convolution with the
symbol built from the oracle's transfer function, element by element, for
every launch-shape variant.

The symbols: which = 1, 1 / C(k h) with C the oracle's shape factor; which
= 2, 1 / K^(k) with the oracle's K^ and, at k = 0, the inverse of the
oracle's (padded) table DC value; k = (2 pi / L) |(a, b)| on the N grid.
Tolerances as for cb_apply_K: FP64 1e-12, FP32 3e-6 relative to max|y|.
"""
import numpy as np
import pytest
import torch

from oracle.transfer import Material, khat, shape_factor, transfer_table

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 3e-6}
DT = {"fp64": torch.float64, "fp32": torch.float32}


def _symbol(N, L, mat, which):
    k = 2 * np.pi * np.fft.fftfreq(N, d=L / N)
    kr = 2 * np.pi * np.fft.rfftfreq(N, d=L / N)
    kk = np.sqrt(k[:, None] ** 2 + kr[None, :] ** 2)
    kk[0, 0] = 1.0
    if which == 1:
        s = 1.0 / shape_factor(kk * mat.h, mat)
        s[0, 0] = 1.0 / float(shape_factor(0.0, mat))
    else:
        s = 1.0 / khat(kk, mat)
        s[0, 0] = 1.0 / transfer_table(N, L, mat)[0, 0]
    return s


def _ref(x, s):
    N = x.shape[0]
    return np.fft.irfft2(np.fft.rfft2(x) * s, s=(N, N))


def _run(lib, N, L, mat, x, prec, which, variant=0):
    plan = lib.cb_plan_create(N, L, mat.h, mat.E1, mat.nu1, mat.E2, mat.nu2, 0.0, prec, fft_variant=variant)
    xt = torch.tensor(x, dtype=DT[prec], device="cuda")
    y = torch.empty_like(xt)
    lib.cb_apply_precond(plan, which, xt, y)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("which", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_precond_random(lib, N, prec, which):
    print(f"precond apply N={N} {prec} which={which}", flush=True)
    mat = Material(0.02, 30.0, 0.3, 1.0, 0.35)
    rng = np.random.default_rng(N + which)
    x = rng.standard_normal((N, N))
    ref = _ref(x, _symbol(N, 1.0, mat, which))
    y = _run(lib, N, 1.0, mat, x, prec, which)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < TOL[prec], f"N={N} {prec} which={which} err={err:.3e}"


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("N", [16, 64, 512])
def test_precond_every_variant(lib, N, variant):
    """Ragged support on the contact-set-like patch, every launch shape."""
    print(f"precond apply variant {variant} N={N}", flush=True)
    mat = Material(0.1, 0.2, 0.25, 1.0, 0.45)
    L = 2.0
    rng = np.random.default_rng(variant)
    x = np.zeros((N, N))
    x[N // 5:N // 2 + 3, N // 3:N - 1] = rng.uniform(-1, 1, (N // 2 + 3 - N // 5, N - 1 - N // 3))
    for prec in ("fp64", "fp32"):
        ref = _ref(x, _symbol(N, L, mat, 2))
        try:
            y = _run(lib, N, L, mat, x, prec, 2, variant)
        except lib.CoatbemError:
            continue   # shape not launchable at this size
        assert np.abs(y - ref).max() / np.abs(ref).max() < TOL[prec]


def test_precond_errors(lib):
    plan = lib.cb_plan_create(64, 1.0, 0.1, 2.0, 0.3, 1.0, 0.3, 0.0, "fp64")
    x = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    for bad in (0, 3, -1):
        with pytest.raises(lib.CoatbemError):
            lib.cb_apply_precond(plan, bad, x, torch.empty_like(x))
