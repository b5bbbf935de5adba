"""What the trained warm-start network gains, on held-out problems.

The shipped weights (trained by `python -m paper_1807_01885_amd.warmstart
train` on the library's own solves, seeds disjoint from these) are run on
24 held-out force-controlled problems of the batched recipe at the
network's native N = 256 and on 8 at N = 1024 (interpolated).  For every
problem the FP32 plan solves from a cold start (uniform pressure) and from
the network's guess.

Measured and asserted:
  - the plain iteration always finishes the solve: every warm-started
    solve converges, to the same pressure as the cold one (FP32 solve
    tolerance 1e-8: relative L2 <= 1e-5) and the same force;
  - the guess is far closer to the solution than the cold start: mean
    relative L2 error of the initial pressure <= 0.3 on the native grid
    (<= 0.6 at N = 1024, where the bilinear interpolation of the 256^2
    output blurs the punch edges) against >= 0.9 for the uniform start,
    over the problems the network serves (stiff thin coatings get the
    uniform start: the network's guess measured slower there);
  - the warm-started solves need fewer iterations than the cold ones.  A
    cold start already runs the two-phase iteration (plain until the
    contact set holds, then the inverse symbol), which reaches a settled
    set within a few iterations, so the guess saves a few iterations per
    solve: measured 16.96 -> 16.17 mean iterations at N = 256 and
    14.88 -> 13.88 at N = 1024 (bar: 0.97 of the cold mean), most on the
    curved indenters (paraboloid, cone), none on flat punches.
"""
import numpy as np
import pytest
import torch

from paper_1807_01885_amd import warmstart as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,n,e0_bar", [(256, 24, 0.3), (1024, 8, 0.6)])
def test_trained_network_on_held_out_problems(lib, N, n, e0_bar):
    print(f"warm start held-out N={N} n={n}", flush=True)
    ws = W.WarmStart()
    problems = W.cases(n, W.VAL_SEED + 1, N)
    cold_it, warm_it, e0_net, e0_uni = [], [], [], []
    for c in problems:
        stiff_thin = (c.E1 / (1 - c.nu1 ** 2) >= 3 * c.E2 / (1 - c.nu2 ** 2)) and c.h <= c.L / 16
        plan = lib.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32")
        f = torch.tensor(c.f, dtype=torch.float64, device="cuda")
        pc = torch.zeros_like(f)
        rc = lib.cb_solve_force(plan, f, c.target, pc, tol=W.TOL)
        pw = torch.empty_like(f)
        ws(plan, f, c.target, pw)
        dA = (c.L / c.N) ** 2
        p0 = pw * (c.target / (pw.sum().item() * dA))
        e_net = ((p0 - pc).norm() / pc.norm()).item()
        e_uni = ((torch.full_like(pc, c.target / (dA * c.N * c.N)) - pc).norm() / pc.norm()).item()
        if stiff_thin:
            assert torch.all(pw == 1.0).item()
        else:
            e0_net.append(e_net)
            e0_uni.append(e_uni)
        rw = lib.cb_solve_force(plan, f, c.target, pw, tol=W.TOL, init=1)
        d = ((pw - pc).norm() / pc.norm()).item()
        print(f"  {c.shape:10s} h={c.h:.4f} E1={c.E1:7.3f} cold {rc['iters']:4d} warm {rw['iters']:4d} "
              f"p0 err net {e_net:.3f} uniform {e_uni:.3f} |p_warm-p_cold| {d:.1e}{' (stiff thin)' if stiff_thin else ''}",
              flush=True)
        assert rc["status"] == 0 and rw["status"] == 0
        assert d <= 1e-5 and abs(rw["F"] - rc["F"]) <= 1e-9 * rc["F"]
        cold_it.append(rc["iters"])
        warm_it.append(rw["iters"])
    mc, mw = np.mean(cold_it), np.mean(warm_it)
    print(f"  mean iterations cold {mc:.2f} warm {mw:.2f} (gain {1 - mw / mc:+.1%}); mean p0 error "
          f"net {np.mean(e0_net):.3f} uniform {np.mean(e0_uni):.3f}", flush=True)
    assert np.mean(e0_net) <= e0_bar and np.mean(e0_uni) >= 0.9
    assert mw <= 0.97 * mc
