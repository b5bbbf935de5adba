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
    output blurs the punch edges) against >= 0.9 for the uniform start;
  - the warm-started solves need far fewer iterations: a caller's guess
    switches the automatic preconditioner to the inverse of the operator's
    symbol, which converges fastest once the contact set is nearly right;
    measured 36.3 -> 18.5 mean iterations at N = 256 and 57.1 -> 14.0 at
    N = 1024; the bar is 0.8 of the cold mean.
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
        plan = lib.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32")
        f = torch.tensor(c.f, dtype=torch.float64, device="cuda")
        pc = torch.zeros_like(f)
        rc = lib.cb_solve_force(plan, f, c.target, pc, tol=W.TOL)
        pw = torch.empty_like(f)
        ws(plan, f, c.target, pw)
        dA = (c.L / c.N) ** 2
        p0 = pw * (c.target / (pw.sum().item() * dA))
        e0_net.append(((p0 - pc).norm() / pc.norm()).item())
        e0_uni.append(((torch.full_like(pc, c.target / (dA * c.N * c.N)) - pc).norm() / pc.norm()).item())
        rw = lib.cb_solve_force(plan, f, c.target, pw, tol=W.TOL, init=1)
        d = ((pw - pc).norm() / pc.norm()).item()
        print(f"  {c.shape:10s} h={c.h:.4f} E1={c.E1:7.3f} cold {rc['iters']:4d} warm {rw['iters']:4d} "
              f"p0 err net {e0_net[-1]:.3f} uniform {e0_uni[-1]:.3f} |p_warm-p_cold| {d:.1e}", flush=True)
        assert rc["status"] == 0 and rw["status"] == 0
        assert d <= 1e-5 and abs(rw["F"] - rc["F"]) <= 1e-9 * rc["F"]
        cold_it.append(rc["iters"])
        warm_it.append(rw["iters"])
    mc, mw = np.mean(cold_it), np.mean(warm_it)
    print(f"  mean iterations cold {mc:.2f} warm {mw:.2f} (gain {1 - mw / mc:+.1%}); mean p0 error "
          f"net {np.mean(e0_net):.3f} uniform {np.mean(e0_uni):.3f}", flush=True)
    assert np.mean(e0_net) <= e0_bar and np.mean(e0_uni) >= 0.9
    assert mw <= 0.8 * mc
