"""cb_apply_K_noalloc (no plan, no allocation) against cb_apply_K.

Two calls in a row on the static intermediate, the second on a smaller
grid, each compared with a plan's cb_apply_K on the same table and input:
FP64 within 1e-12, FP32 within 3e-6 of max |u| (the apply bars).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

MAT = (0.05, 10.0, 0.3, 1.0, 0.25)  # h, E1, nu1, E2, nu2


def _table(lib, N, L, prec):
    h, E1, nu1, E2, nu2 = MAT
    T, _ = lib.cb_transfer_table(N, L, h, E1, nu1, E2, nu2)
    T = T * (1.0 / (2.0 * N * 2.0 * N))
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.tensor(T, dtype=torch.float64, device="cuda").to(dt).contiguous()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_apply_K(lib, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    L = 1.0
    h, E1, nu1, E2, nu2 = MAT
    rng = np.random.default_rng(11)
    for N in (1024, 128):
        print(f"noalloc {prec} N={N}", flush=True)
        p = torch.tensor(rng.standard_normal((N, N)), dtype=dt, device="cuda")
        table = _table(lib, N, L, prec)
        u0 = torch.full((N, N), float("nan"), dtype=dt, device="cuda")
        lib.cb_apply_K_noalloc(N, prec, table, p, u0)
        plan = lib.cb_plan_create(N, L, h, E1, nu1, E2, nu2, 0.0, prec)
        u1 = torch.empty_like(p)
        lib.cb_apply_K(plan, p, u1)
        torch.cuda.synchronize()
        a, b = u0.double().cpu().numpy(), u1.double().cpu().numpy()
        err = np.abs(a - b).max() / np.abs(b).max()
        print(f"  max rel diff {err:.2e}")
        assert np.isfinite(a).all()
        assert err <= (1e-12 if prec == "fp64" else 3e-6)


def test_noalloc_rejects_beyond_scratch(lib):
    t = torch.zeros(2049, 2049, dtype=torch.float64, device="cuda")
    p = torch.zeros(2048, 2048, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(p)
    with pytest.raises(lib.CoatbemError) as ei:
        lib.cb_apply_K_noalloc(2048, "fp64", t, p, u)
    assert ei.value.status == lib.CB_E_INVALID
