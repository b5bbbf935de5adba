"""Learned warm start of the constrained conjugate-gradient contact solve.

A small U-Net (see include/coatbem.h, "Learned warm start") maps the
indenter profile and the problem scalars (h/L, E1/E2, nu1, nu2, load) on a
256 x 256 grid to an initial pressure field.  This module generates its
training data with the library's own solves, trains it with the library's
own BF16 matrix-core forward/backward kernels and Adam, stores the weights
(plain .npy + JSON, no pickle) and applies it.  The solve always finishes
from the guess with the plain method and its own convergence test, so the
network changes the iteration count, never the answer.

    python -m paper_1807_01885_amd.warmstart train --out DIR
    python -m paper_1807_01885_amd.warmstart evaluate --weights DIR/warmstart_g256.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import coatbem as cb
from . import inputs

G = 256
C = 16
NLAYER = 12
HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "warmstart_g256.npy")
TRAIN_SEED = 20240
VAL_SEED = 31337
TOL = 1e-8


def init_params(seed):
    """He-normal weights (std sqrt(2 / (9 C))), zero biases, head scaled by 0.1."""
    n = cb.cb_net_num_params()
    lp = n // NLAYER
    rng = np.random.default_rng(seed)
    p = np.zeros(n, dtype=np.float32)
    for l in range(NLAYER):
        std = math.sqrt(2.0 / (9 * C)) * (0.1 if l == NLAYER - 1 else 1.0)
        p[l * lp:l * lp + 9 * C * C] = rng.standard_normal(9 * C * C) * std
    return p


def cases(n, seed, N=G):
    """Force-controlled problems of the batched recipe on one grid size."""
    return inputs.batch_c4(n=n, seed=seed, N_choices=(N,), adhesion=False)


@dataclass
class Dataset:
    N: int
    f: torch.Tensor                       # (n, N, N) float64, device
    t: torch.Tensor                       # (n, N, N) float32, device: solved pressure
    scal: list = field(default_factory=list)   # (L, h, E1, nu1, E2, nu2, F) per sample
    iters: list = field(default_factory=list)  # cold-start iterations of the solve

    def __len__(self):
        return len(self.scal)


def generate(problems, chunk=64, workers=0, tol=TOL, log=print):
    """Solve every problem (FP32 plans, cold start) and keep (f, p)."""
    N = problems[0].N
    n = len(problems)
    f_all = torch.empty((n, N, N), dtype=torch.float64, device="cuda")
    t_all = torch.empty((n, N, N), dtype=torch.float32, device="cuda")
    keep, scal, iters = [], [], []
    t0 = time.time()
    for s in range(0, n, chunk):
        part = problems[s:s + chunk]
        plans = [cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, "fp32") for c in part]
        fs = [torch.tensor(c.f, dtype=torch.float64, device="cuda") for c in part]
        ps = [torch.zeros_like(x) for x in fs]
        res = cb.cb_solve_batch(plans, fs, [c.target for c in part], [1] * len(part), ps,
                                workers=workers, raise_on_error=False, tol=tol)
        for j, (c, r) in enumerate(zip(part, res)):
            if r["status"] != cb.CB_OK:
                continue
            k = len(keep)
            f_all[k] = fs[j]
            t_all[k] = ps[j].float()
            keep.append(s + j)
            scal.append((c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, c.target))
            iters.append(r["iters"])
        log(f"  solved {min(s + chunk, n)}/{n} ({time.time() - t0:.1f} s)")
    k = len(keep)
    return Dataset(N, f_all[:k], t_all[:k], scal, iters)


def _features(net, ds, idx, x):
    for j, i in enumerate(idx):
        cb.cb_net_features(net, ds.f[i], *ds.scal[i], x[j])


def evaluate_loss(net, ds, batch):
    x = torch.empty((batch, net.H, net.W, C), dtype=torch.float32, device="cuda")
    tot, cnt = 0.0, 0
    for s in range(0, len(ds), batch):
        idx = list(range(s, min(s + batch, len(ds))))
        _features(net, ds, idx, x)
        loss = cb.cb_net_loss_grad(net, x[:len(idx)], ds.t[idx].contiguous())
        tot += loss * len(idx)
        cnt += len(idx)
    return tot / cnt


def train(ds, steps=4000, batch=16, lr=2e-3, seed=0, val=None, log=print, log_every=200):
    """Adam with linear warm-up and cosine decay; returns (params, history)."""
    g = ds.N  # the network is trained on the grid of its data
    net = cb.cb_net_create(batch, g, g)
    cb.cb_net_set_params(net, torch.tensor(init_params(seed), device="cuda"))
    rng = np.random.default_rng(seed)
    x = torch.empty((batch, g, g, C), dtype=torch.float32, device="cuda")
    hist = []
    run = 0.0
    t0 = time.time()
    warm = max(1, steps // 40)
    for it in range(1, steps + 1):
        idx = rng.choice(len(ds), size=batch, replace=False)
        _features(net, ds, idx, x)
        loss = cb.cb_net_loss_grad(net, x, ds.t[torch.as_tensor(idx, device="cuda")].contiguous())
        a = min(1.0, it / warm)
        cur = lr * a * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / steps)))
        cb.cb_net_adam_step(net, cur)
        run = loss if it == 1 else 0.98 * run + 0.02 * loss
        if it % log_every == 0 or it == steps:
            rec = {"step": it, "train": run, "lr": cur, "s": time.time() - t0}
            if val is not None:
                rec["val"] = evaluate_loss(net, val, batch)
            hist.append(rec)
            log("  " + " ".join(f"{k} {v:.4g}" if isinstance(v, float) else f"{k} {v}" for k, v in rec.items()))
    return cb.cb_net_get_params(net).cpu().numpy(), hist


def save(params, path, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)
    with open(os.path.splitext(path)[0] + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)


def load(path=WEIGHTS):
    params = np.load(path, allow_pickle=False)
    if params.shape != (cb.cb_net_num_params(),) or params.dtype != np.float32:
        raise ValueError(f"{path}: expected {cb.cb_net_num_params()} float32 parameters")
    meta = {}
    mp = os.path.splitext(path)[0] + ".json"
    if os.path.exists(mp):
        with open(mp) as fh:
            meta = json.load(fh)
    return params, meta


class WarmStart:
    """Trained network bound to a stream: ws(plan, f, F, p_out) fills p_out."""

    def __init__(self, path=WEIGHTS, cut=None, stream=None, params=None, batch=1, grid=None):
        meta = {}
        if params is None:
            params, meta = load(path)
        self.meta = meta
        self.cut = float(meta.get("cut", 0.1) if cut is None else cut)
        self.grid = int(meta.get("grid", G) if grid is None else grid)
        self.net = cb.cb_net_create(batch, self.grid, self.grid, stream=stream)
        cb.cb_net_set_params(self.net, torch.tensor(params, device="cuda"))

    def __call__(self, plan, f, F, p_out):
        return cb.cb_net_warmstart(self.net, plan, f, F, p_out, cut=self.cut)

    def batch(self, plans, fs, Fs, ps_out):
        """Warm starts of up to `batch` problems with one forward pass."""
        return cb.cb_net_warmstart_batch(self.net, plans, fs, Fs, ps_out, cut=self.cut)


def compare(ws, problems, tol=TOL, precision="fp32", log=None):
    """Cold and warm solve of each problem: iterations and the relative L2
    difference of the two converged pressures."""
    rows = []
    for c in problems:
        plan = cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu1, c.E2, c.nu2, 0.0, precision)
        f = torch.tensor(c.f, dtype=torch.float64, device="cuda")
        p_cold = torch.zeros_like(f)
        rc = cb.cb_solve_force(plan, f, c.target, p_cold, tol=tol)
        p_warm = torch.empty_like(f)
        ws(plan, f, c.target, p_warm)
        p0 = p_warm.clone()
        rw = cb.cb_solve_force(plan, f, c.target, p_warm, tol=tol, init=1)
        diff = ((p_warm - p_cold).norm() / p_cold.norm()).item()
        s0 = p0.sum().item()
        # no guess (zeros: stiff thin coatings) -> the warm solve is the cold one
        err0 = (((p0 * (c.target / (s0 * (c.L / c.N) ** 2)) - p_cold).norm() / p_cold.norm()).item()
                if s0 > 0 else float("nan"))
        row = {"shape": c.shape, "N": c.N, "cold": rc["iters"], "warm": rw["iters"], "diff": diff, "p0_err": err0,
               "ms_cold": rc["ms"], "ms_warm": rw["ms"]}
        rows.append(row)
        if log:
            log(f"  {c.shape:10s} N={c.N} cold {rc['iters']:4d} warm {rw['iters']:4d} p0 err {err0:.3f} diff {diff:.1e}")
    return rows


def _choose_cut(params, grid, problems, cuts, log):
    best = None
    for cut in cuts:
        rows = compare(WarmStart(cut=cut, params=params, grid=grid), problems)
        m = float(np.mean([r["warm"] for r in rows]))
        log(f"  cut {cut:g}: mean warm iterations {m:.2f} (cold {np.mean([r['cold'] for r in rows]):.2f})")
        if best is None or m < best[1]:
            best = (cut, m)
    return best[0]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--n-train", type=int, default=4096)
    tr.add_argument("--n-val", type=int, default=256)
    tr.add_argument("--steps", type=int, default=4000)
    tr.add_argument("--batch", type=int, default=16)
    tr.add_argument("--lr", type=float, default=2e-3)
    tr.add_argument("--seed", type=int, default=0)
    tr.add_argument("--out", default=os.path.dirname(WEIGHTS))
    tr.add_argument("--grid", type=int, default=G, help="network grid = grid of the training solves")
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", default=WEIGHTS)
    ev.add_argument("--n", type=int, default=32)
    ev.add_argument("--N", type=int, default=G)
    ev.add_argument("--seed", type=int, default=VAL_SEED + 1)
    a = ap.parse_args(argv)

    def log(s):
        print(s, flush=True)

    if a.cmd == "train":
        log(f"generating {a.n_train} training and {a.n_val} validation solves at N={a.grid}")
        ds = generate(cases(a.n_train, TRAIN_SEED, a.grid), log=log)
        val = generate(cases(a.n_val, VAL_SEED, a.grid), log=log)
        log(f"training {a.steps} steps, batch {a.batch}")
        params, hist = train(ds, a.steps, a.batch, a.lr, a.seed, val=val, log=log)
        meta = {"grid": a.grid, "cut": 0.2, "n_train": len(ds), "n_val": len(val), "steps": a.steps,
                "batch": a.batch, "lr": a.lr, "seed": a.seed, "train_seed": TRAIN_SEED, "val_seed": VAL_SEED,
                "tol": TOL, "final": hist[-1], "cold_iters_mean": float(np.mean(ds.iters))}
        path = os.path.join(a.out, f"warmstart_g{a.grid}.npy")
        save(params, path, meta)  # kept before the cut is chosen
        del ds, val
        meta["cut"] = _choose_cut(params, a.grid, cases(48, VAL_SEED + 7, a.grid), (0.03, 0.1, 0.2, 0.35), log)
        save(params, path, meta)
        log(f"saved {path} (cut {meta['cut']})")
    else:
        ws = WarmStart(a.weights)
        rows = compare(ws, cases(a.n, a.seed, a.N), log=log)
        c = np.mean([r["cold"] for r in rows])
        w = np.mean([r["warm"] for r in rows])
        log(f"mean iterations cold {c:.2f} warm {w:.2f} (gain {1 - w / c:.1%}); "
            f"max |p_warm - p_cold| / |p_cold| {max(r['diff'] for r in rows):.1e}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
