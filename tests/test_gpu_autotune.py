"""FFT launch-shape variants and the autotuner.

Every variant is the same transform with a different thread/tile shape, so
each must meet the apply parity bar against the FP64 oracle (FP64 1e-12,
FP32 3e-6 relative to max|u|, as for the default shape).  The tuner must
pick a fitting variant, record its time, write one cache line and reuse
it; a solve on a tuned plan converges to the same pressure."""
import os

import numpy as np
import pytest
import torch

from oracle.operator import Operator
from oracle.transfer import Material
from paper_1807_01885_amd import inputs

pytestmark = pytest.mark.gpu

LAYER_M = Material(0.05, 20.0, 0.3, 1.0, 0.25)
LAYER = (LAYER_M.h, LAYER_M.E1, LAYER_M.nu1, LAYER_M.E2, LAYER_M.nu2)
TOL = {"fp64": 1e-12, "fp32": 3e-6}
DT = {"fp64": torch.float64, "fp32": torch.float32}
NVAR = 6


@pytest.mark.parametrize("N", [16, 64, 256, 1024, 2048, 4096])
def test_every_variant_matches_oracle(lib, N):
    print(f"variants N={N}", flush=True)
    rng = np.random.default_rng(N + 11)
    p = rng.standard_normal((N, N))
    ref = Operator(N, 1.0, LAYER_M).apply(p)
    scale = np.abs(ref).max()
    for prec in ("fp64", "fp32"):
        pt = torch.tensor(p, dtype=DT[prec], device="cuda")
        for v in range(1, NVAR + 1):
            try:
                plan = lib.cb_plan_create(N, 1.0, *LAYER, 0.0, prec, fft_variant=v)
            except lib.CoatbemError as e:
                # only a shape too large for one block (LDS or 1024 threads)
                # at the largest size may be refused
                assert e.status == lib.CB_E_UNSUPPORTED and N >= 2048, str(e)
                print(f"  {prec} variant {v}: not launchable at this size", flush=True)
                continue
            assert lib.cb_plan_get_info(plan)["fft_variant"] == v
            u = torch.empty_like(pt)
            lib.cb_apply_K(plan, pt, u)
            torch.cuda.synchronize()
            err = np.abs(u.double().cpu().numpy() - ref).max() / scale
            print(f"  {prec} variant {v}: {err:.2e}", flush=True)
            assert err < TOL[prec], f"N={N} {prec} variant {v} err={err:.3e}"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotune_and_cache(lib, prec, tmp_path):
    print(f"autotune {prec}", flush=True)
    cache = str(tmp_path / "tune.txt")
    N = 512
    plan = lib.cb_plan_create(N, 1.0, *LAYER, 0.0, prec, autotune=1, tune_cache=cache)
    info = lib.cb_plan_get_info(plan)
    assert 1 <= info["fft_variant"] <= NVAR and info["tune_us"] > 0.0
    print(f"  chose variant {info['fft_variant']} at {info['tune_us']:.2f} us", flush=True)
    lines = [l for l in open(cache).read().split("\n") if l.strip()]
    # FP32 plans also tune the FP64 convolutions that refresh u in the solvers
    assert len(lines) == (1 if prec == "fp64" else 2)
    arch, n, pr, v, us = lines[0].split()
    assert int(n) == N and int(pr) == (0 if prec == "fp64" else 1) and int(v) == info["fft_variant"] - 1
    if prec == "fp32":
        assert lines[1].split()[2] == "0"
    # a second tuned plan reads the cache instead of timing again
    plan2 = lib.cb_plan_create(N, 1.0, *LAYER, 0.0, prec, autotune=1, tune_cache=cache)
    info2 = lib.cb_plan_get_info(plan2)
    assert info2["fft_variant"] == info["fft_variant"] and info2["tune_us"] == pytest.approx(float(us))
    assert len([l for l in open(cache).read().split("\n") if l.strip()]) == len(lines)
    # without autotune the cache entry is still used
    plan3 = lib.cb_plan_create(N, 1.0, *LAYER, 0.0, prec, tune_cache=cache)
    assert lib.cb_plan_get_info(plan3)["fft_variant"] == info["fft_variant"]
    # and without either, the built-in shape
    plan4 = lib.cb_plan_create(N, 1.0, *LAYER, 0.0, prec)
    assert lib.cb_plan_get_info(plan4)["fft_variant"] == 1 and lib.cb_plan_get_info(plan4)["tune_us"] == 0.0
    # a tuned plan solves to the same pressure as the default one
    f = torch.tensor(inputs.paraboloid(N, 1.0, 1.0), dtype=torch.float64, device="cuda")
    pa, pb = torch.zeros_like(f), torch.zeros_like(f)
    tol = 1e-10 if prec == "fp64" else 1e-8
    lib.cb_solve_force(plan, f, 2e-3, pa, tol=tol)
    lib.cb_solve_force(plan4, f, 2e-3, pb, tol=tol)
    diff = ((pa - pb).norm() / pb.norm()).item()
    assert diff < (1e-8 if prec == "fp64" else 1e-5), diff


def test_variant_option_errors(lib):
    for kw in ({"fft_variant": NVAR + 1}, {"fft_variant": -1}, {"autotune": 2}):
        with pytest.raises(lib.CoatbemError) as e:
            lib.cb_plan_create(64, 1.0, *LAYER, 0.0, "fp32", **kw)
        assert e.value.status == lib.CB_E_INVALID
    # a cache path that cannot be written does not fail the plan
    plan = lib.cb_plan_create(64, 1.0, *LAYER, 0.0, "fp32", autotune=1,
                              tune_cache=os.path.join("/nonexistent-dir", "t.txt"))
    assert lib.cb_plan_get_info(plan)["tune_us"] > 0.0
