"""GPU parity of cb_apply_K (u = K p, Eq. 11 on the 2N-padded grid) against
the FP64 oracle, element by element.

Tolerances: FP64 1e-12 relative to max|u| (rounding of ~log2(M) FFT
stages); FP32 (FP32 FFT with FP64-derived tables) 3e-6 relative to
max|u|, derived from eps32 * (log2 M passes + twiddle rounding).
"""
import numpy as np
import pytest
import torch

from oracle.operator import Operator
from oracle.transfer import Material

pytestmark = pytest.mark.gpu

LAYER = Material(0.1, 10.0, 0.3, 1.0, 0.3)
TOL = {"fp64": 1e-12, "fp32": 3e-6}
DT = {"fp64": torch.float64, "fp32": torch.float32}


def _run(lib, N, L, mat, p, prec):
    plan = lib.cb_plan_create(N, L, mat.h, mat.E1, mat.nu1, mat.E2, mat.nu2, 0.0, prec)
    pt = torch.tensor(p, dtype=DT[prec], device="cuda")
    u = torch.empty_like(pt)
    lib.cb_apply_K(plan, pt, u)
    torch.cuda.synchronize()
    return plan, u.double().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_apply_random(lib, N, prec):
    print(f"apply random N={N} {prec}", flush=True)
    rng = np.random.default_rng(N + (0 if prec == "fp64" else 7))
    p = rng.standard_normal((N, N))
    op = Operator(N, 1.0, LAYER)
    ref = op.apply(p)
    _, u = _run(lib, N, 1.0, LAYER, p, prec)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err < TOL[prec], f"N={N} {prec} err={err:.3e}"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mat", [Material(0.02, 0.1, 0.25, 1.0, 0.45),
                                 Material(0.0, 2.0, 0.3, 2.0, 0.3),
                                 Material(5.0, 0.05, 0.45, 1.0, 0.2)])
def test_apply_materials_and_ragged_support(lib, mat, prec):
    """Pressure on an off-centre rectangle touching the grid edges."""
    N, L = 256, 2.0
    rng = np.random.default_rng(3)
    p = np.zeros((N, N))
    p[0:77, 131:N] = rng.uniform(0, 1, (77, N - 131))
    op = Operator(N, L, mat)
    ref = op.apply(p)
    _, u = _run(lib, N, L, mat, p, prec)
    assert np.abs(u - ref).max() / np.abs(ref).max() < TOL[prec]


def test_apply_zero_and_determinism(lib):
    N = 128
    plan = lib.cb_plan_create(N, 1.0, 0.1, 10.0, 0.3, 1.0, 0.3, 0.0, "fp64")
    z = torch.zeros(N, N, dtype=torch.float64, device="cuda")
    u = torch.full_like(z, 7.0)
    lib.cb_apply_K(plan, z, u)
    torch.cuda.synchronize()
    assert torch.count_nonzero(u).item() == 0
    p = torch.rand(N, N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    u1 = torch.empty_like(p)
    u2 = torch.empty_like(p)
    lib.cb_apply_K(plan, p, u1)
    lib.cb_apply_K(plan, p, u2)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)


@pytest.mark.parametrize("N", [128, 1024])
def test_apply_fp32_deterministic(lib, N):
    plan = lib.cb_plan_create(N, 1.0, 0.1, 10.0, 0.3, 1.0, 0.3, 0.0, "fp32")
    g = torch.Generator("cuda").manual_seed(2)
    p = torch.rand(N, N, dtype=torch.float32, device="cuda", generator=g)
    us = [torch.empty_like(p) for _ in range(4)]
    for u in us:
        lib.cb_apply_K(plan, p, u)
    torch.cuda.synchronize()
    for u in us[1:]:
        assert torch.equal(us[0], u)


def test_apply_on_side_stream(lib):
    N = 64
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = lib.cb_plan_create(N, 1.0, 0.1, 10.0, 0.3, 1.0, 0.3, 0.0, "fp64")
        p = torch.ones(N, N, dtype=torch.float64, device="cuda")
        u = torch.empty_like(p)
        lib.cb_apply_K(plan, p, u)
    s.synchronize()
    ref = Operator(N, 1.0, LAYER).apply(np.ones((N, N)))
    assert np.abs(u.cpu().numpy() - ref).max() / ref.max() < 1e-12


def test_plan_table_matches_oracle(lib):
    N, L = 128, 1.0
    plan = lib.cb_plan_create(N, L, 0.1, 10.0, 0.3, 1.0, 0.3, 1e-3, "fp32")
    T = lib.cb_plan_get_table(plan)
    from oracle.transfer import transfer_table, critical_stress
    ref = transfer_table(N, L, LAYER)[: N + 1, : N + 1]
    np.testing.assert_allclose(T, ref, rtol=1e-11)
    info = lib.cb_plan_get_info(plan)
    assert info["sigma_c"] == pytest.approx(critical_stress(LAYER, 1e-3, L / N), rel=1e-14)
    assert info["M"] == 2 * N and info["precision"] == 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N,n", [(64, 40), (256, 9), (1024, 3)])
def test_apply_batch_equals_individual(lib, N, n, prec):
    """cb_apply_K_batch packs n problems (different coatings, one size) into
    one launch per stage (groups of 32): each output equals the problem's
    own cb_apply_K bit for bit (same kernels, tables and arithmetic), and
    the first matches the oracle (1e-12 FP64, 3e-6 FP32 of max |u|)."""
    print(f"apply batch N={N} n={n} {prec}", flush=True)
    from oracle.operator import Operator
    from oracle.transfer import Material
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(N + n)
    mats = [Material(float(rng.uniform(0.01, 0.2)), float(rng.uniform(0.05, 50.0)), 0.3, 1.0,
                     float(rng.uniform(0.2, 0.45))) for _ in range(n)]
    plans = [lib.cb_plan_create(N, 1.0, m.h, m.E1, m.nu1, m.E2, m.nu2, 0.0, prec) for m in mats]
    ps = [torch.tensor(rng.standard_normal((N, N)), dtype=dt, device="cuda") for _ in range(n)]
    us = [torch.full((N, N), float("nan"), dtype=dt, device="cuda") for _ in range(n)]
    lib.cb_apply_K_batch(plans, ps, us)
    torch.cuda.synchronize()
    for i in range(n):
        u1 = torch.empty_like(ps[i])
        lib.cb_apply_K(plans[i], ps[i], u1)
        torch.cuda.synchronize()
        assert torch.equal(u1, us[i]), f"problem {i} differs from its own apply"
    op = Operator(N, 1.0, mats[0])
    ref = op.apply(ps[0].double().cpu().numpy())
    err = np.abs(us[0].double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= (1e-12 if prec == "fp64" else 3e-6)


def test_apply_batch_rejects_mixed(lib):
    a = lib.cb_plan_create(64, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3, 0.0, "fp64")
    b = lib.cb_plan_create(128, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3, 0.0, "fp64")
    c = lib.cb_plan_create(64, 1.0, 0.1, 1.0, 0.3, 1.0, 0.3, 0.0, "fp64", kernel_mode="periodic")
    p64 = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    p128 = torch.zeros(128, 128, dtype=torch.float64, device="cuda")
    for plans, ps in (([a, b], [p64, p128]), ([a, c], [p64, p64.clone()])):
        with pytest.raises(lib.CoatbemError) as e:
            lib.cb_apply_K_batch(plans, ps, [torch.empty_like(x) for x in ps])
        assert e.value.status == lib.CB_E_INVALID
