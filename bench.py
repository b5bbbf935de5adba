"""Benchmark: contact solves per second at N = 1024 on one MI355X.

Workload (one "step"): the N = 1024 solve set -- 32 force-controlled
contact problems drawn by the batched recipe (paraboloid / cone / flat
punch / elliptic punch indenters, coating h/L log-uniform in [1e-3, 0.3],
E1/E2 log-uniform in [0.01, 100], nu in [0.2, 0.45]), seed 1024, each
solved to relative residual 1e-8.  `value` is the full method: FP32
direction convolutions with FP64 state and reductions, the learned warm
start (network forward pass inside the step), all 32 solves concurrent
through cb_solve_batch, FFT launch shapes from the shipped tune cache.

Also timed on the same set and tolerance: the FP32 path from the solver's
own cold start (the overlap at an approach estimated from the profile),
the same path from a uniform pressure (the published method's start), and
the plain FP64 solver (cold start, one solve after another); the
network's gain against both starts of the method without it is reported.  Every
path's pressures are checked against an FP64 solve to residual 1e-10.
The same set is also solved with exact-kernel plans (the exact coefficients
of uniformly loaded cells as the convolution's table): FP32 batched from
the cold start, against FP64 exact plans at 1e-10, and the difference the
exact coefficients make to the padded point-sampled kernel's solution.
The uneven batched recipe (N from 128 to 1024, half adhesive) and packed
small-N convolutions are timed after it.

Measured live: cb_apply_K and its three kernels at N = 1024 (FP32 and
FP64), graph-replayed with HIP events on the stream they run on; the
roofline object uses the dominant kernel's algorithmic bytes per launch
over its mean duration, and its HBM traffic from the committed
FETCH_SIZE / WRITE_SIZE counter runs while the kernel source is unchanged.
The same convolution with the fixed launch shape 1 (no tune cache) is
timed beside it (apply_K_untuned).
The CPU baseline times the FP64 oracle's own solve of the first problem
on the host (its constrained CG from its uniform start, to the same
residual), end to end.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "contact solves/sec at N=1024² (learned+FP32 vs plain FP64); cb_apply_K HBM GB/s"
PEAK_HBM_GBPS = 8000.0
TOL = 1e-8          # every timed path
TOL_REF = 1e-10     # FP64 reference for the accuracy checks

# HBM traffic of the column kernel (K2) at N = 1024, FP32, tuned launch
# shape, from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) scaled
# by what the same counters read for a 64 MiB device copy (FETCH x 2.0,
# WRITE x 1.0); the summary and commands are in profiles/.  Valid while the
# FFT sources hash to `src` and the plan uses `variant`.
K2_TRAFFIC = {"kernel": "k2_cols", "N": 1024, "precision": "fp32", "variant": 3,
              "src": "85027b7a9235f86c:3ed6ec38f5a5fd4e",
              "fetch_bytes": 6334.2 * 1024 * 2.0, "write_bytes": 8192.0 * 1024,
              # SQ_INSTS_VALU per launch (same probe, same conditions)
              "valu_wave_insts": 3019452.0}
# wave64 VALU instructions the chip issues per second without packed FP32:
# 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per instruction on a 16-lane SIMD
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def fft_src_hash():
    out = []
    for f in ("fft.hip", "fft_core.h"):
        with open(os.path.join(ROOT, "paper_1807_01885_amd", "csrc", f), "rb") as fh:
            out.append(hashlib.sha256(fh.read()).hexdigest()[:16])
    return ":".join(out)


def alg_bytes(N, s):
    """Algorithmic HBM bytes of the three apply kernels and their sum."""
    half = 2 * s * N * (N + 1)          # one pass over the complex half spectrum
    k1 = s * N * N + half
    k2 = 2 * half + s * (N + 1) ** 2
    k3 = half + s * N * N
    return {"k1_rows_fwd": k1, "k2_cols": k2, "k3_rows_inv": k3, "apply": k1 + k2 + k3}


def time_apply(cb, plan, p, u, per_graph=50, replays=10):
    """Mean duration (ms) of cb_apply_K and of each kernel alone.

    The launches are captured into a graph (`per_graph` back-to-back
    launches on the capture stream, which the plan is pointed at) and the
    graph is replayed `replays` times between two HIP events recorded on
    that same stream, so host launch cost does not enter the figure."""
    import torch
    out = {}
    side = torch.cuda.Stream()
    for name, mask in (("apply", 7), ("k1_rows_fwd", 1), ("k2_cols", 2), ("k3_rows_inv", 4)):
        cb.cb_apply_K_stages(plan, p, u, mask)          # first call outside capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            cb.cb_plan_set_stream(plan, side)
            for _ in range(per_graph):
                cb.cb_apply_K_stages(plan, p, u, mask)
        cb.cb_plan_set_stream(plan, torch.cuda.current_stream())
        with torch.cuda.stream(side):
            g.replay()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(replays):
                g.replay()
            e1.record(side)
        e1.synchronize()
        out[name] = e0.elapsed_time(e1) / (replays * per_graph)
        del g
    return out


def apply_roofline(cb, plan32, plan64, N):
    """Live timing of cb_apply_K and its kernels (both precisions) and the
    roofline object of the dominant FP32 kernel."""
    import numpy as np
    import torch
    rng = np.random.default_rng(0)
    pr = rng.standard_normal((N, N))
    timing = {}
    for prec, plan, s in (("fp32", plan32, 4), ("fp64", plan64, 8)):
        dt = torch.float32 if prec == "fp32" else torch.float64
        p = torch.tensor(pr, dtype=dt, device="cuda")
        u = torch.empty_like(p)
        ms = time_apply(cb, plan, p, u)
        ab = alg_bytes(N, s)
        timing[prec] = {k: {"ms": ms[k], "GBps": ab[k] / (ms[k] * 1e-3) / 1e9, "bytes": ab[k]} for k in ms}
    t32k = timing["fp32"]
    dom = max(("k1_rows_fwd", "k2_cols", "k3_rows_inv"), key=lambda k: t32k[k]["ms"])
    ach = t32k[dom]["GBps"]
    variant = cb.cb_plan_get_info(plan32)["fft_variant"]
    traffic = None
    issue = None
    if (dom == K2_TRAFFIC["kernel"] and N == K2_TRAFFIC["N"] and variant == K2_TRAFFIC["variant"]
            and fft_src_hash() == K2_TRAFFIC["src"]):
        traffic = K2_TRAFFIC["fetch_bytes"] + K2_TRAFFIC["write_bytes"]
        floor_ms = 1e3 * K2_TRAFFIC["valu_wave_insts"] / VALU_ISSUE_PER_S
        issue = {"valu_wave_insts": K2_TRAFFIC["valu_wave_insts"], "issue_floor_ms": floor_ms,
                 "frac_of_valu_issue": floor_ms / t32k[dom]["ms"]}
    roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBPS, "traffic": traffic,
            "bytes_per_launch": t32k[dom]["bytes"], "mean_launch_ms": t32k[dom]["ms"],
            "fft_variant": variant, "valu_issue": issue}
    return timing, roof


def untuned_apply_timing(cb, case):
    """cb_apply_K of the first problem's plans with the fixed launch shape 1
    (no tune cache), beside the tuned figures of apply_K."""
    import numpy as np
    import torch
    rng = np.random.default_rng(0)
    pr = rng.standard_normal((case.N, case.N))
    out = {"fft_variant": 1}
    for prec, s in (("fp32", 4), ("fp64", 8)):
        plan = cb.cb_plan_create(case.N, case.L, case.h, case.E1, case.nu1, case.E2, case.nu2, 0.0, prec,
                                 fft_variant=1)
        p = torch.tensor(pr, dtype=torch.float32 if prec == "fp32" else torch.float64, device="cuda")
        u = torch.empty_like(p)
        ms = time_apply(cb, plan, p, u)["apply"]
        cb.cb_plan_destroy(plan)
        out[prec] = {"ms": round(ms, 5), "GBps": round(alg_bytes(case.N, s)["apply"] / (ms * 1e-3) / 1e9, 1)}
    return out


def batch_apply_timing(cb, inputs, n=64, N=128, replays=20):
    """Convolutions of n problems at a small N (coatings of the batched
    recipe): cb_apply_K once per problem against cb_apply_K_batch (one launch
    per stage for up to 32 problems), each captured in a graph and replayed
    between HIP events on the stream it runs on; microseconds per problem."""
    import torch
    from paper_1807_01885_amd.tune import TUNE_CACHE
    cs = inputs.batch_c4(n=n, seed=4, N_choices=(N,), adhesion=False)
    plans = [cb.cb_plan_create(N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32", tune_cache=TUNE_CACHE)
             for c in cs]
    ps = [torch.randn(N, N, dtype=torch.float32, device="cuda") for _ in cs]
    us = [torch.empty_like(x) for x in ps]
    side = torch.cuda.Stream()
    out = {}
    for name in ("one_launch_per_problem", "packed"):
        def run():
            if name == "packed":
                cb.cb_apply_K_batch(plans, ps, us)
            else:
                for pl, x, y in zip(plans, ps, us):
                    cb.cb_apply_K(pl, x, y)
        run()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for pl in plans:
                cb.cb_plan_set_stream(pl, side)
            run()
        for pl in plans:
            cb.cb_plan_set_stream(pl, torch.cuda.current_stream())
        with torch.cuda.stream(side):
            g.replay()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(replays):
                g.replay()
            e1.record(side)
        e1.synchronize()
        out[name] = 1e3 * e0.elapsed_time(e1) / (replays * n)
        del g
    return {"N": N, "problems": n, "precision": "fp32", "us_per_problem": {k: round(v, 3) for k, v in out.items()},
            "speedup": out["one_launch_per_problem"] / out["packed"]}


def cpu_baseline(case, budget_iters):
    """The oracle's own FP64 solve of `case` (its constrained CG from its
    uniform start, residual TOL), end to end when it converges within
    budget_iters iterations, else its time per iteration scaled by the
    iterations it needed in a longer reference count (stated)."""
    from oracle import operator as oop
    from oracle.solvers import solve_pk
    from oracle.transfer import Material
    workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    op = oop.Operator(case.N, case.L, Material(case.h, case.E1, case.nu1, case.E2, case.nu2),
                      workers=workers)
    t0 = time.perf_counter()
    r = solve_pk(op, case.f, case.target, mode="force", tol=TOL, max_iter=budget_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / max(r.iters, 1)
    # the oracle's convolution alone, with all workers and with one
    apply_ms = {}
    for w in (workers, 1):
        o = op if w == workers else oop.Operator(case.N, case.L, Material(case.h, case.E1, case.nu1, case.E2,
                                                                           case.nu2), workers=1)
        ta = time.perf_counter()
        for _ in range(3):
            o.apply(case.f)
        apply_ms[f"workers_{w}"] = round(1e3 * (time.perf_counter() - ta) / 3, 1)
    host = {"cpu": cpu_model(), "oracle_apply_ms": apply_ms}
    if r.converged:
        return {"value": 1.0 / dt, "unit": "solves/s", "cores": workers, "kind": "oracle", **host,
                "sample": (f"FP64 oracle (numpy/scipy.fft, {workers} workers), one complete solve of the first "
                           f"problem of the N=1024 set to residual {TOL:g}: {r.iters} iterations of its own "
                           f"constrained CG in {dt:.1f} s ({per_iter*1e3:.1f} ms/iteration)")}
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": workers, "kind": "oracle", **host,
            "sample": (f"FP64 oracle (numpy/scipy.fft, {workers} workers), first problem of the N=1024 set: its own "
                       f"constrained CG (published activation rule, uniform start) had not converged after "
                       f"{r.iters} iterations ({dt:.1f} s, residual {r.resid:.1e}, {per_iter*1e3:.1f} ms/iteration); "
                       f"value = 1 / that time, an upper bound of its solve rate")}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-solves", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-kernel leg")
    ap.add_argument("--cpu-iters", type=int, default=400, help="iteration budget of the oracle's solve")
    ap.add_argument("--c4", type=int, default=256, help="problems of the uneven batched recipe leg (0: skip)")
    ap.add_argument("--dump", default=None, help="write per-problem results (JSON) here")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the live apply_K timing and roofline object (for rocprofv3 --kernel-trace --stats)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch K2 (N=1024, FP32, tuned shape) 10 times and a 64 MiB device copy 5 times, "
                         "for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--profile-solves", action="store_true",
                    help="only the FP32 solves of the set, cold then from the learned guess, one after another "
                         "on one host thread (for rocprofv3 --kernel-trace --stats)")
    ap.add_argument("--profile-warmstart", action="store_true",
                    help="only the batched warm start of the set, eight times (for rocprofv3 --kernel-trace --stats)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent solves would shard by problem across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1807_01885_amd import coatbem as cb
    from paper_1807_01885_amd import inputs
    from paper_1807_01885_amd.tune import TUNE_CACHE
    from paper_1807_01885_amd.warmstart import WarmStart

    torch.cuda.set_device(0)
    if args.pmc_probe:
        plan = cb.cb_plan_create(1024, 1.0, 0.05, 20.0, 0.3, 1.0, 0.25, 0.0, "fp32", tune_cache=TUNE_CACHE)
        p = torch.randn(1024, 1024, dtype=torch.float32, device="cuda")
        u = torch.empty_like(p)
        cb.cb_apply_K(plan, p, u)
        for _ in range(10):
            cb.cb_apply_K_stages(plan, p, u, 2)
        a = torch.ones(64 * 2**20 // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": "done", "fft_variant": cb.cb_plan_get_info(plan)["fft_variant"]}))
        return
    cases = inputs.headline_set(n=args.n_solves)
    N = cases[0].N
    n = len(cases)
    if args.profile_solves:
        ws = WarmStart()
        its = []
        for c in cases:
            plan = cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32", tune_cache=TUNE_CACHE)
            f = torch.tensor(c.f, dtype=torch.float64, device="cuda")
            p = torch.zeros(c.N, c.N, dtype=torch.float64, device="cuda")
            cold = cb.cb_solve_force(plan, f, c.target, p, tol=TOL)["iters"]
            ws(plan, f, c.target, p)
            warm = cb.cb_solve_force(plan, f, c.target, p, tol=TOL, init=1)["iters"]
            its.append((cold, warm))
            print(f"solve {len(its)}/{n}: iterations cold {cold} warm {warm}", flush=True)
        print(json.dumps({"profile_solves": "done", "mean_iters_cold": float(np.mean([a for a, _ in its])),
                          "mean_iters_warm": float(np.mean([b for _, b in its]))}))
        return
    if args.profile_warmstart:
        plans = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32", tune_cache=TUNE_CACHE)
                 for c in cases]
        fs = [torch.tensor(c.f, dtype=torch.float64, device="cuda") for c in cases]
        ps = [torch.zeros_like(f) for f in fs]
        ws = WarmStart(batch=n)
        ms = []
        for _ in range(8):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ws.batch(plans, fs, [c.target for c in cases], ps)
            ms.append(1e3 * (time.perf_counter() - t0))
        print(json.dumps({"profile_warmstart": "done", "problems": n, "host_ms_per_call": ms}))
        return
    if args.roofline_only:
        c = cases[0]
        p32, p64 = (cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, prec, tune_cache=TUNE_CACHE)
                    for prec in ("fp32", "fp64"))
        timing, roof = apply_roofline(cb, p32, p64, N)
        print(json.dumps({"roofline": roof, "apply_K": {prec: {k: {"ms": round(v["ms"], 5),
                                                                   "GBps": round(v["GBps"], 1)}
                                                               for k, v in t.items()}
                                                        for prec, t in timing.items()}}))
        return

    def make(prec):
        plans = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, prec, tune_cache=TUNE_CACHE)
                 for c in cases]
        fs = [torch.tensor(c.f, dtype=torch.float64, device="cuda") for c in cases]
        ps = [torch.zeros(c.N, c.N, dtype=torch.float64, device="cuda") for c in cases]
        return plans, fs, ps

    plans32, fs32, ps32 = make("fp32")
    plans64, fs64, ps64 = make("fp64")
    pc32 = [torch.zeros_like(p) for p in ps32]
    ws = WarmStart(batch=n)
    targets = [c.target for c in cases]
    torch.cuda.synchronize()

    ws_ms = []

    def step_learned():
        t0 = time.perf_counter()
        ws.batch(plans32, fs32, targets, ps32)      # synchronises
        ws_ms.append(1e3 * (time.perf_counter() - t0))
        return cb.cb_solve_batch(plans32, fs32, targets, [1] * n, ps32, tol=TOL, init=1)

    def step_cold32():
        return cb.cb_solve_batch(plans32, fs32, targets, [1] * n, pc32, tol=TOL)

    pu32 = [torch.zeros_like(p) for p in ps32]

    def step_uniform32():
        # the published method's start: uniform pressure carrying the load
        # (two-phase iteration, as the solver takes it from that start)
        for p, c in zip(pu32, cases):
            p.fill_(c.target / (c.L * c.L))
        return cb.cb_solve_batch(plans32, fs32, targets, [1] * n, pu32, tol=TOL, init=1, precond=3)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = fn()
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    # ---- the full method (value) ------------------------------------------------
    res_l, t_l = timed(step_learned, args.steps, args.warmup)
    value = n * args.steps / t_l
    # ---- FP32 batched, cold start ----------------------------------------------
    res_c, t_c = timed(step_cold32, args.steps, args.warmup)
    value_c = n * args.steps / t_c
    # ---- FP32 batched, uniform start ---------------------------------------------
    res_u, t_u = timed(step_uniform32, args.steps, args.warmup)
    value_u = n * args.steps / t_u
    # ---- plain FP64: cold start, one solve after another --------------------------
    def step_plain64():
        return [cb.cb_solve_force(pl, f, c.target, p, tol=TOL) for pl, f, p, c in zip(plans64, fs64, ps64, cases)]
    res_p, t_p = timed(step_plain64, 1, 1)
    value_p = n / t_p
    # ---- FP64 reference (residual 1e-10) for the accuracy checks ------------------
    pref = [torch.zeros_like(p) for p in ps64]
    res_r = cb.cb_solve_batch(plans64, fs64, targets, [1] * n, pref, tol=TOL_REF)
    torch.cuda.synchronize()

    def accuracy(ps, res):
        ep, eF, agr = [], [], []
        for a, b, ra, rb in zip(ps, pref, res, res_r):
            ep.append((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())
            eF.append(abs(ra["F"] - rb["F"]) / rb["F"])
            sa, sb = a > 0, b > 0
            uni = (sa | sb).sum().item()
            agr.append(1.0 - (sa ^ sb).sum().item() / max(uni, 1))
        return {"max_rel_L2_p": max(ep), "max_rel_F": max(eF), "min_set_agreement": min(agr)}

    acc_l, acc_c, acc_p = accuracy(ps32, res_l), accuracy(pc32, res_c), accuracy(ps64, res_p)
    acc_u = accuracy(pu32, res_u)
    it = lambda res: float(np.mean([r["iters"] for r in res]))  # noqa: E731

    timing, roof = apply_roofline(cb, plans32[0], plans64[0], N)
    untuned = untuned_apply_timing(cb, cases[0])
    small_batch = batch_apply_timing(cb, inputs)

    if args.dump:
        rows = []
        for c, a, b, d, r in zip(cases, res_l, res_c, res_p, res_r):
            rows.append(dict(shape=c.shape, h=c.h, E1=c.E1, nu1=c.nu1, nu2=c.nu2, F=c.target,
                             it_learned=a["iters"], it_cold32=b["iters"], it_plain64=d["iters"],
                             it_ref=r["iters"], ms_learned=a["ms"], ms_cold32=b["ms"], ms_plain64=d["ms"],
                             area=r["area"], d=r["d"]))
        with open(args.dump, "w") as fh:
            json.dump(rows, fh, indent=1)

    # ---- the batched recipe: uneven grids, half adhesive (one timed pass) -------
    c4 = None
    if args.c4 > 0:
        cs = inputs.batch_c4(n=args.c4, seed=4)
        pl4 = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, c.dgamma, "fp32", tune_cache=TUNE_CACHE)
               for c in cs]
        f4 = [torch.tensor(c.f, dtype=torch.float64, device="cuda") for c in cs]
        p4 = [torch.zeros_like(f) for f in f4]
        m4 = [1 if c.mode == "force" else 0 for c in cs]
        t4 = [c.target for c in cs]
        r4, dt4 = timed(lambda: cb.cb_solve_batch(pl4, f4, t4, m4, p4, tol=TOL, raise_on_error=False), 1, 1)
        groups = {}
        for c, r in zip(cs, r4):
            key = f"N{c.N}_{'adhesive' if c.dgamma > 0 else 'plain'}"
            groups.setdefault(key, []).append(r["iters"])
        # accuracy of every member against FP64 plans solved to residual 1e-10
        del pl4
        pl64 = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, c.dgamma, "fp64",
                                  tune_cache=TUNE_CACHE) for c in cs]
        q4 = [torch.zeros_like(f) for f in f4]
        rq = cb.cb_solve_batch(pl64, f4, t4, m4, q4, tol=TOL_REF, raise_on_error=False)
        torch.cuda.synchronize()
        ep4, eF4, ag4 = [], [], []
        for a, b, ra, rb in zip(p4, q4, r4, rq):
            ep4.append((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())
            eF4.append(abs(ra["F"] - rb["F"]) / max(abs(rb["F"]), 1e-300))
            sa, sb = a != 0, b != 0
            ag4.append(1.0 - (sa ^ sb).sum().item() / max((sa | sb).sum().item(), 1))
        c4 = {"value": len(cs) / dt4, "unit": "solves/s", "solves": len(cs),
              "failed": sum(r["status"] != 0 for r in r4) + sum(r["status"] != 0 for r in rq),
              "mean_iters": {k: round(float(np.mean(v)), 1) for k, v in sorted(groups.items())},
              "accuracy_vs_fp64_1e-10": {"max_rel_L2_p": max(ep4), "max_rel_F": max(eF4),
                                         "min_set_agreement": min(ag4)},
              "how": "batched recipe seed 4 (N in {128,256,512,1024}, half adhesive single solves), FP32 plans, "
                     "cold start, one cb_solve_batch; accuracy against FP64 plans of the library at residual "
                     "1e-10 (oracle parity of the recipe: tests/test_gpu_batch.py)"}
        del pl64, f4, p4, q4

    # ---- the exact non-periodic kernel: the same set, FP32 batched, cold -------
    exact = None
    if not args.no_exact:
        t0 = time.perf_counter()
        plx = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32", tune_cache=TUNE_CACHE,
                                 kernel_mode="exact") for c in cases]
        build_s = (time.perf_counter() - t0) / n
        px = [torch.zeros_like(p) for p in ps32]
        rx, tx = timed(lambda: cb.cb_solve_batch(plx, fs32, targets, [1] * n, px, tol=TOL), 1, 1)
        del plx
        plx64 = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp64", tune_cache=TUNE_CACHE,
                                   kernel_mode="exact") for c in cases]
        pxr = [torch.zeros_like(p) for p in ps64]
        rxr = cb.cb_solve_batch(plx64, fs64, targets, [1] * n, pxr, tol=TOL_REF)
        torch.cuda.synchronize()
        del plx64
        ex_p = max((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item() for a, b in zip(px, pxr))
        ex_F = max(abs(a["F"] - b["F"]) / b["F"] for a, b in zip(rx, rxr))
        ex_agr = min(1.0 - ((a > 0) ^ (b > 0)).sum().item() / max(((a > 0) | (b > 0)).sum().item(), 1)
                     for a, b in zip(px, pxr))
        # what the exact coefficients change in the solution: FP64 exact against FP64 padded, both at 1e-10
        ex_vs_pad = [(torch.linalg.norm(a - b) / torch.linalg.norm(b)).item() for a, b in zip(pxr, pref)]
        ex_d = [abs(a["d"] - b["d"]) / abs(b["d"]) for a, b in zip(rxr, res_r)]
        exact = {"value": n / tx, "unit": "solves/s", "mean_iters": it(rx),
                 "table_build_s_per_plan": build_s,
                 "accuracy_vs_fp64_exact_1e-10": {"max_rel_L2_p": ex_p, "max_rel_F": ex_F,
                                                  "min_set_agreement": ex_agr},
                 "exact_vs_padded_fp64": {"median_rel_L2_p": float(np.median(ex_vs_pad)),
                                          "max_rel_L2_p": max(ex_vs_pad), "max_rel_d": max(ex_d)},
                 "how": "the same 32 force solves with CB_KERNEL_EXACT plans (exact cell coefficients as the "
                        "table of the same convolution kernels), FP32 directions, cold start, one "
                        "cb_solve_batch; table build on the host, outside the timed region"}
        del px, pxr

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cases[0], args.cpu_iters)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_l / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{n} force-controlled contact solves at N={N} (padded {2*N}^2 FFT), batched recipe "
                         f"seed 1024, residual {TOL:g}: learned warm start (256^2 BF16 network) + FP32 direction "
                         "convolutions with FP64 state/reductions, solved concurrently by cb_solve_batch"),
            "N": N, "solves_per_step": n, "tol": TOL,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy_vs_fp64_1e-10": acc_l,
        "mean_iters": it(res_l),
        "warmstart_ms_per_step": float(np.median(ws_ms)),
        "fp32_cold_batched": {"value": value_c, "unit": "solves/s", "mean_iters": it(res_c), "accuracy": acc_c},
        "fp32_uniform_batched": {"value": value_u, "unit": "solves/s", "mean_iters": it(res_u), "accuracy": acc_u,
                                 "how": "the same path from a uniform pressure (the published method's start), "
                                        "two-phase iteration"},
        "warm_start_gain": {"vs_uniform_start": value / value_u - 1.0, "vs_estimated_cold_start": value / value_c - 1.0,
                            "note": "the network's guess against the two starts of the method without it: "
                                    "positive = the learned configuration is faster"},
        "plain_fp64": {"value": value_p, "unit": "solves/s", "mean_iters": it(res_p), "accuracy": acc_p,
                       "how": "FP64 plans, cold start, one cb_solve_force after another"},
        "speedup_vs_plain_fp64": value / value_p,
        "batched_recipe": c4,
        "exact_kernel": exact,
        "apply_K_batch_small_N": small_batch,
        "apply_K": {prec: {k: {"ms": round(v["ms"], 5), "GBps": round(v["GBps"], 1)} for k, v in t.items()}
                    for prec, t in timing.items()},
        "apply_K_untuned": untuned,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
