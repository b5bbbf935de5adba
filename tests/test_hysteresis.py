"""Approach/retraction hysteresis maps over (alpha, E1/E2)
(paper_1807_01885_amd/hysteresis.py): the case construction on the CPU;
on the GPU, the batched map against single sweeps, the loop closing as
the work of adhesion vanishes, and the pull-off force of the two limits the
paper gives, homogeneous JKR (-3/2 pi R dgamma) and the thin layer on a
rigid base (Eq. 19: -2 pi R dgamma)."""
import math

import numpy as np
import pytest
import torch

from oracle import analytic as an


def test_case_construction():
    from paper_1807_01885_amd import hysteresis as hy
    for alpha, ratio in [(0.1, 1.0), (0.5, 1.0), (2.0, 0.1), (2.0, 10.0), (15.0, 1e-5)]:
        c = hy.make_case(alpha, ratio)
        E1s, E2s = c.E1 / (1 - c.nu ** 2), c.E2 / (1 - c.nu ** 2)
        assert an.adhesion_parameter(c.dgamma, c.R, E1s, c.h) == pytest.approx(alpha, rel=1e-12)
        assert c.E1 / c.E2 == pytest.approx(ratio, rel=1e-12)
        D = c.L / c.N
        # a0: JKR's radius at zero load with the softer modulus
        a0 = (9 * math.pi * c.dgamma * c.R ** 2 / (2 * min(E1s, E2s))) ** (1 / 3)
        F0, _ = an.jkr(a0, c.R, min(E1s, E2s), c.dgamma)
        assert abs(F0) <= 1e-12 * math.pi * c.R * c.dgamma
        assert D <= c.h / 8 + 1e-15 and c.N * D >= 5.2 * a0 and c.N & (c.N - 1) == 0
        d = c.d_steps
        na = c.n_approach
        step = d[0]
        # the approach rises on a lattice and the retraction comes back on it
        assert np.allclose(np.diff(d[:na]), step, rtol=1e-12)
        assert np.allclose(np.diff(d[na - 1:]), -step, rtol=1e-12)
        assert np.any(d[na:] == 0.0)
        _, _, dJ = an.jkr_pulloff_displacement_control(c.R, min(E1s, E2s), c.dgamma)
        assert d[-1] <= 3 * dJ + 1e-15 and d[-1] > 3 * dJ - step
    with pytest.raises(ValueError):
        hy.make_case(15.0, 1e-5, max_N=256)


def test_summary_of_records():
    """The loop work is the trapezoid rule over the recorded path from the
    origin, the pull-off figures come from the last step in contact."""
    from paper_1807_01885_amd import hysteresis as hy
    c = hy.make_case(0.5, 1.0, approach_steps=2)
    c.d_steps = np.array([1.0, 2.0, 1.0, 0.0, -1.0, -2.0])
    c.n_approach = 2
    F = [1.0, 3.0, 1.5, -0.5, -1.0, 0.0]
    A = [0.5, 1.0, 0.8, 0.4, 0.1, 0.0]
    recs = [dict(d=x, F=y, area=z, rounds=1, status=0) for x, y, z in zip(c.d_steps, F, A)]
    s = hy.summarise(c, recs)
    W = 0.5 * 1 + 2.0 * 1 + 2.25 * -1 + 0.5 * -1 + -0.75 * -1 + -0.5 * -1
    assert s["W_loop"] == pytest.approx(W, abs=1e-15)
    assert s["W_approach"] == pytest.approx(0.5 + 2.0, abs=1e-15)
    assert s["F_min"] == -1.0 and s["d_last"] == -1.0 and s["lost"]
    assert s["a_last"] == pytest.approx(math.sqrt(0.1 / math.pi), rel=1e-15)
    assert s["a_max"] == pytest.approx(math.sqrt(1.0 / math.pi), rel=1e-15)


@pytest.mark.gpu
def test_map_equals_single_sweeps(lib):
    """The batched map is orchestration only: every case equals its own
    cb_sweep bit for bit."""
    from paper_1807_01885_amd import hysteresis as hy
    cases = [hy.make_case(al, ra, approach_steps=40) for al in (0.2, 2.0) for ra in (0.1, 10.0)]
    print("map cases N", [c.N for c in cases], flush=True)
    summ = hy.run_cases(cases, "fp32")
    for c, s in zip(cases, summ):
        plan = lib.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu, c.E2, c.nu, c.dgamma, "fp32")
        f = torch.tensor(hy.inputs.paraboloid(c.N, c.L, c.R), dtype=torch.float64, device="cuda")
        p = torch.zeros_like(f)
        m = torch.zeros(c.N, c.N, dtype=torch.uint8, device="cuda")
        rec = lib.cb_sweep(plan, f, c.d_steps, p, m, tol=1e-8)
        lib.cb_plan_destroy(plan)
        assert all(r["status"] == 0 for r in rec)
        assert np.array_equal(s["F"], [r["F"] for r in rec]) and np.array_equal(s["area"], [r["area"] for r in rec])
        print(f"  alpha {c.alpha:g} E1/E2 {c.ratio:g} N {c.N}: F_min / (pi R dgamma) "
              f"{s['F_min'] / (math.pi * c.R * c.dgamma):.3f}, W_loop / W_approach {s['W_loop'] / s['W_approach']:.3f}, "
              f"lost {s['lost']}", flush=True)
        assert s["lost"] and s["d_last"] < 0.0 and s["F_min"] < 0.0
        assert s["W_loop"] > 0.01 * s["W_approach"]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hysteresis_vanishes_with_adhesion(lib, prec):
    """The cycle dissipates through adhesion: with the work of adhesion
    scaled down 1000 times on the same geometry, grid and steps, the
    loop's net work relative to the approach work falls far below the
    adhesive case's (in JKR the dissipation goes as dgamma^(5/3) at a fixed
    approach), and the retraction retraces the approach: the force at each
    approach met on both branches agrees to 2% of the largest force."""
    from paper_1807_01885_amd import hysteresis as hy
    full, weak = hy.run_cases([hy.make_case(0.5, 10.0, approach_steps=40),
                               hy.make_case(0.5, 10.0, approach_steps=40, dgamma_scale=1e-3)], prec)
    rf, rw = full["W_loop"] / full["W_approach"], weak["W_loop"] / weak["W_approach"]
    na = full["n_approach"]
    step = full["d"][0]
    back = {round(x / step): y for x, y in zip(weak["d"][na:], weak["F"][na:])}
    err = max(abs(back[round(x / step)] - y) for x, y in zip(weak["d"][:na - 1], weak["F"][:na - 1]))
    print(f"  W_loop / W_approach: dgamma {rf:.3e}, dgamma / 1000 {rw:.3e}; branches of the weak case apart "
          f"by {err / weak['F'].max():.1e} of F_max", flush=True)
    assert rf > 0.01 and abs(rw) <= 0.05 * rf
    assert err <= 0.02 * weak["F"].max()


@pytest.mark.gpu
@pytest.mark.parametrize("alpha,ratio,factor", [(0.5, 1.0, 1.5), (15.0, 1e-5, 2.0)])
def test_pulloff_force_limits(lib, alpha, ratio, factor):
    """Most tensile force of the displacement-controlled cycle: the
    homogeneous case (E1 = E2) at JKR's -3/2 pi R dgamma, a thin layer on a
    rigid base at large alpha at Eq. 19's -2 pi R dgamma; bars 10%."""
    from paper_1807_01885_amd import hysteresis as hy
    c = hy.make_case(alpha, ratio)
    print(f"alpha {alpha:g}, E1/E2 {ratio:g}: N {c.N}, D = h/{c.h / (c.L / c.N):.2f}", flush=True)
    s = hy.run_cases([c], "fp32")[0]
    assert all(st == 0 for st in s["status"])
    q = s["F_min"] / (-factor * math.pi * c.R * c.dgamma)
    print(f"  F_min / (-{factor:g} pi R dgamma) = {q:.4f}; last contact d = {s['d_last']:.4g} a = {s['a_last']:.4g}; "
          f"W_loop / W_approach {s['W_loop'] / s['W_approach']:.3f}", flush=True)
    assert abs(q - 1.0) <= 0.10
    assert s["lost"] and s["W_loop"] > 0.0
