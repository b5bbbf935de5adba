"""Adhesive approach/retraction hysteresis of a paraboloid on a coated
half-space, mapped over the adhesion parameter alpha (Eq. 26) and the
stiffness ratio E1/E2.

Each case is the quasi-static procedure of Sec. 2 (last paragraph): the
rigid approach d grows in equal steps to d_max and then falls on the same
lattice until the contact is lost, every step solved with the detachment
criterion of Eq. 12.  The cases run as concurrent sweeps on the GPU
(cb_sweep_batch); this module only builds the cases and reduces the
per-step records.

Units: layer thickness h = 1 and E1 = 1; nu1 = nu2 = nu; the work of
adhesion is dgamma = g * E1 * h with g = 5e-5 by default (the ratio of
the paper's Fig. 5 example: 100 J/m^2 on a 2 mm layer of 1 GPa).  alpha
fixes the radius, R = alpha * sqrt(E1* h^3 / (2 dgamma)) (Eq. 26 solved
for R).

Grid: the sizes come from the JKR relations of the softer of the two
materials (modulus E* = min(E1*, E2*)), which bound the contact from above:
zero-load radius a0^3 = 9 pi dgamma R^2 / (2 E*) and displacement-control
pull-off approach d_J = -3 a_c^2 / R with a_c^3 = pi dgamma R^2 / (8 E*).
Cells are D = min(h / cells_per_h, a0 / cells_per_a0): below h, as Eq. 12
needs, and fine against the contact.  N is the smallest power of two with
N D >= span * a0 (at least min_N).  The approach runs to
d_max = (1.3 a0)^2 / R in `approach_steps` steps; the retraction continues
on the same lattice to -3 |d_J|.

Summary of each case (from the per-step records of the library):
  F_min          most tensile force of the sweep (the pull-off force
                 under displacement control)
  d_last, a_last approach and equivalent radius sqrt(area / pi) at the
                 last step in contact on the way out
  lost           whether the contact was lost before the last step
  a_max          largest equivalent radius (at d_max)
  W_loop         net work of the indenter over the cycle,
                 sum over steps of (F_k + F_{k-1}) / 2 * (d_k - d_{k-1})
                 from d = 0, F = 0: the energy the cycle dissipates (it
                 vanishes with the work of adhesion)
  W_approach     the same sum over the approach alone
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import coatbem as cb
from . import inputs


@dataclass
class HysteresisCase:
    alpha: float
    ratio: float           # E1 / E2
    nu: float
    h: float
    E1: float
    E2: float
    dgamma: float
    R: float
    N: int
    L: float
    d_steps: np.ndarray = field(repr=False)
    n_approach: int = 0


def make_case(alpha, ratio, nu=0.3, g=5e-5, approach_steps=80, cells_per_h=8, cells_per_a0=24,
              span=5.2, min_N=128, max_N=2048, dgamma_scale=1.0):
    """One case of the map (see the module docstring).  dgamma_scale
    multiplies the work of adhesion of the plan and keeps the geometry,
    grid and steps of the case."""
    if not (alpha > 0 and ratio > 0 and 0 <= nu < 0.5 and g > 0 and approach_steps >= 2 and dgamma_scale > 0):
        raise ValueError("alpha, ratio, g and dgamma_scale must be positive, 0 <= nu < 0.5, approach_steps >= 2")
    h, E1 = 1.0, 1.0
    E2 = E1 / ratio
    E1s, E2s = E1 / (1 - nu * nu), E2 / (1 - nu * nu)
    dg = g * E1 * h
    R = alpha * math.sqrt(E1s * h ** 3 / (2.0 * dg))
    Es = min(E1s, E2s)
    a0 = (9.0 * math.pi * dg * R * R / (2.0 * Es)) ** (1.0 / 3.0)
    ac = (math.pi * dg * R * R / (8.0 * Es)) ** (1.0 / 3.0)
    dJ = 3.0 * ac * ac / R
    D = min(h / cells_per_h, a0 / cells_per_a0)
    N = min_N
    while N * D < span * a0:
        N *= 2
    if N > max_N:
        raise ValueError(f"alpha = {alpha}, E1/E2 = {ratio}: the contact needs N = {N} > {max_N} cells")
    dstep = (1.3 * a0) ** 2 / R / approach_steps
    n_back = approach_steps + int(math.ceil(3.0 * dJ / dstep))
    k = np.concatenate([np.arange(1, approach_steps + 1), approach_steps - np.arange(1, n_back + 1)])
    return HysteresisCase(alpha=alpha, ratio=ratio, nu=nu, h=h, E1=E1, E2=E2, dgamma=dg * dgamma_scale,
                          R=R, N=N, L=N * D, d_steps=k * dstep, n_approach=approach_steps)


def summarise(case, records):
    """Branches and summary figures of one swept case (module docstring)."""
    d = np.array([r["d"] for r in records])
    F = np.array([r["F"] for r in records])
    area = np.array([r["area"] for r in records])
    a = np.sqrt(area / math.pi)
    dd = np.diff(np.concatenate([[0.0], d]))
    Fm = 0.5 * (F + np.concatenate([[0.0], F[:-1]]))
    work = Fm * dd
    na = case.n_approach
    out = dict(alpha=case.alpha, ratio=case.ratio, R=case.R, h=case.h, dgamma=case.dgamma, N=case.N, L=case.L,
               d=d, F=F, area=area, a=a, rounds=np.array([r["rounds"] for r in records]), n_approach=na,
               status=[r["status"] for r in records])
    contact = np.nonzero(area[na:] > 0.0)[0]
    last = na + contact[-1] if len(contact) else na - 1
    out.update(F_min=float(F.min()), d_last=float(d[last]), a_last=float(a[last]), a_max=float(a.max()),
               lost=bool(area[-1] == 0.0), W_loop=float(work.sum()), W_approach=float(work[:na].sum()))
    return out


def hysteresis_map(alphas, ratios, precision="fp32", workers=0, tol=None, **case_opts):
    """Sweeps of every (alpha, E1/E2) pair, run concurrently; returns one
    summary dict per case (alphas outer, ratios inner)."""
    cases = [make_case(al, ra, **case_opts) for al in alphas for ra in ratios]
    return run_cases(cases, precision=precision, workers=workers, tol=tol)


def run_cases(cases, precision="fp32", workers=0, tol=None):
    """Sweep the given cases with cb_sweep_batch and summarise them."""
    if tol is None:
        tol = 1e-8 if precision == "fp32" else 1e-10
    plans = []
    try:
        for c in cases:
            plans.append(cb.cb_plan_create(c.N, c.L, c.h, c.E1, c.nu, c.E2, c.nu, c.dgamma, precision))
        fs = [torch.tensor(inputs.paraboloid(c.N, c.L, c.R), dtype=torch.float64, device="cuda") for c in cases]
        ps = [torch.zeros_like(f) for f in fs]
        ms = [torch.zeros(c.N, c.N, dtype=torch.uint8, device="cuda") for c in cases]
        recs = cb.cb_sweep_batch(plans, fs, [c.d_steps for c in cases], ps, ms, workers=workers, tol=tol)
    finally:
        for pl in plans:
            cb.cb_plan_destroy(pl)
    return [summarise(c, r) for c, r in zip(cases, recs)]
