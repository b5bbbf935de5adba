"""Inverse problems on the coated half-space (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Sec. 2, paragraph after Eq. 11: the pressure producing a prescribed
    displacement is found by conjugate gradients ([8], the BEM of Pohrt and
    Popov for the homogeneous half-space).  [8] is not in the paper; the
    reading adopted is the constrained conjugate-gradient method of
    Polonsky and Keer (Wear 231, 1999), which is the standard scheme behind
    [8].  Its converged result is the unique solution of the linear
    complementarity problem
        p >= 0,  g = K p + f - d >= 0,  p . g = 0
    (K is symmetric positive definite), which `solve_nnls` computes by an
    independent route on tiny grids.
  * Sec. 2, Eq. 12 and the last paragraph of Sec. 2: adhesive contact.
    Elements at the boundary of the contact detach when their tensile
    stress exceeds sigma_c; the stress is recomputed on the reduced area
    and the check repeated until no boundary element exceeds sigma_c;
    then the next displacement step.

Readings adopted where the paper is silent:
  * sign conventions: f >= 0 is the indenter profile, d the rigid
    approach (positive into the body), p > 0 compressive, u the surface
    displacement into the body, F = Delta^2 sum p;
  * detachment is simultaneous for every violating boundary cell; the
    boundary is the set of contact cells with a 4-neighbour outside the
    contact or on the grid edge; cells outside the contact that
    penetrate the indenter attach; a cell detached within a displacement
    step does not re-attach within that step;
  * a single adhesive solve (no history) starts from the geometric
    overlap {f <= d}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.optimize

from .operator import Operator


@dataclass
class SolveResult:
    p: np.ndarray
    u: np.ndarray
    d: float
    iters: int
    resid: float
    converged: bool
    F: float = 0.0
    area: float = 0.0
    history: list = field(default_factory=list)


def self_influence(op: Operator) -> float:
    """Displacement of a cell under unit pressure on itself (kernel at 0)."""
    e = np.zeros((op.N, op.N))
    e[0, 0] = 1.0
    return float(op.apply(e)[0, 0])


# ---------------------------------------------------------------------------
# Non-adhesive contact: constrained conjugate gradients (Polonsky-Keer)
# ---------------------------------------------------------------------------
def solve_pk(op: Operator, f, target, mode="disp", p0=None, tol=1e-10,
             max_iter=20000):
    """Non-adhesive normal contact by constrained conjugate gradients.

    mode "disp": target is the rigid approach d; mode "force": target is
    the total force F = Delta^2 sum p and d is returned.

    Iteration (one K-application of p and one of the direction t):
      g = u + f - d on the current contact set Ic = {p > 0}; force control
      replaces d by the mean of u + f over Ic;  G = sum_Ic g^2;
      t = g + delta (G/G_old) t on Ic, 0 elsewhere;  r = K t (mean over Ic
      removed in force control);  tau = sum_Ic g t / sum_Ic r t;
      p <- max(p - tau t, 0);  cells with p = 0 and g < 0 get p <- -tau g
      and reset delta to 0 (else delta = 1);  force control rescales p to F.
    When the direction carries no energy (sum_Ic r t = 0, e.g. a single
    active cell already exact) tau falls back to 1/K_00 so that the
    penetrating cells still enter with the local (self-influence) estimate.
    Stops when the relative residual ||g||_Ic / ||d - f||_Ic <= tol and
    no cell with p = 0 penetrates (g < -tol * rms(d - f)_Ic).
    """
    f = np.asarray(f, dtype=np.float64)
    dA = op.dx ** 2
    force = mode == "force"
    if force:
        F = float(target)
        d = 0.0
        if F <= 0.0:
            z = np.zeros_like(f)
            return SolveResult(z, z.copy(), float(f.min()), 0, 0.0, True)
    else:
        d = float(target)
        if d <= f.min():
            z = np.zeros_like(f)
            return SolveResult(z, z.copy(), d, 0, 0.0, True)
    if p0 is not None:
        p = np.maximum(np.asarray(p0, dtype=np.float64), 0.0)
    elif force:
        p = np.full_like(f, F / (dA * f.size))
    else:
        p = np.maximum(d - f, 0.0) / self_influence(op)
    k00 = self_influence(op)
    if force:
        p *= F / (dA * p.sum())

    t = np.zeros_like(f)
    G_old = 1.0
    delta = 0.0
    res = math.inf
    converged = False
    it = 0
    u = op.apply(p)
    d_eff = d
    for it in range(1, max_iter + 1):
        Ic = p > 0.0
        g = u + f - d
        if force:
            gbar = g[Ic].mean()
            g -= gbar
            d_eff = gbar
        rhs = (d_eff - f)[Ic]
        rnorm = math.sqrt(float(np.dot(rhs, rhs)))
        gn = math.sqrt(float(np.dot(g[Ic], g[Ic])))
        res = gn / rnorm if rnorm > 0 else gn
        scale = rnorm / math.sqrt(max(int(Ic.sum()), 1))
        viol = int(np.count_nonzero((~Ic) & (g < -tol * scale)))
        if res <= tol and viol == 0:
            converged = True
            break
        G = gn * gn
        beta = delta * G / G_old if delta > 0.0 else 0.0
        t = np.where(Ic, g + beta * t, 0.0)
        G_old = G
        r = op.apply(t)
        if force:
            r -= r[Ic].mean()
        rt = float(np.dot(r[Ic], t[Ic]))
        tau = float(np.dot(g[Ic], t[Ic])) / rt if rt > 0.0 else 1.0 / k00
        p = np.where(Ic, p - tau * t, p)
        p = np.maximum(p, 0.0)
        Iol = (p == 0.0) & (g < 0.0)
        if Iol.any():
            delta = 0.0
            p[Iol] -= tau * g[Iol]
        else:
            delta = 1.0
        if force:
            p *= F / (dA * p.sum())
        u = op.apply(p)
    return SolveResult(p, u, d_eff, it, res, converged,
                       F=dA * float(p.sum()), area=dA * float((p > 0).sum()))


# ---------------------------------------------------------------------------
# Brute force for tiny grids: the LCP as a non-negative least-squares problem
# ---------------------------------------------------------------------------
def solve_nnls(op: Operator, f, d):
    """Minimise 1/2 p.K p - p.(d - f) over p >= 0 with K = R^T R (Cholesky).

    Equivalent to NNLS  min ||R p - b||, R^T b = d - f; its KKT conditions
    are exactly the complementarity problem of the contact.
    """
    K = op.dense_matrix()
    R = scipy.linalg.cholesky(K, lower=False)
    rhs = (d - np.asarray(f, dtype=np.float64)).ravel()
    b = scipy.linalg.solve_triangular(R, rhs, trans="T", lower=False)
    p, _ = scipy.optimize.nnls(R, b, maxiter=50 * K.shape[0])
    return p.reshape(op.N, op.N)


def solve_nnls_force(op: Operator, f, F):
    """Force control by bisection on d of the brute-force solution."""
    dA = op.dx ** 2
    f = np.asarray(f, dtype=np.float64)
    lo = float(f.min())
    hi = lo + 1e-3 * op.L
    while dA * solve_nnls(op, f, hi).sum() < F:
        hi = lo + 2.0 * (hi - lo)
    d = scipy.optimize.brentq(lambda dd: dA * solve_nnls(op, f, dd).sum() - F,
                              lo, hi, xtol=1e-15 * op.L, rtol=1e-15)
    return solve_nnls(op, f, d), d


# ---------------------------------------------------------------------------
# Adhesive contact (Eq. 12 and the pull-off procedure of Sec. 2)
# ---------------------------------------------------------------------------
def solve_on_set(op: Operator, f, d, S, p0=None, tol=1e-10, max_iter=20000):
    """Pressure on a fixed contact set S: (K p)_i = d - f_i on S, p = 0 off S.

    Plain conjugate gradients on the symmetric positive definite block
    K_SS; the sign of p is free (adhesive tension allowed).  Returns
    (p, iterations, relative residual).
    """
    f = np.asarray(f, dtype=np.float64)
    b = np.where(S, d - f, 0.0)
    bn = math.sqrt(float(np.dot(b.ravel(), b.ravel())))
    if not S.any() or bn == 0.0:
        return np.zeros_like(f), 0, 0.0
    x = np.zeros_like(f) if p0 is None else np.where(S, p0, 0.0)
    r = b - np.where(S, op.apply(x), 0.0)
    z = r.copy()
    rr = float(np.dot(r.ravel(), r.ravel()))
    it = 0
    for it in range(1, max_iter + 1):
        if math.sqrt(rr) <= tol * bn:
            break
        q = np.where(S, op.apply(z), 0.0)
        alpha = rr / float(np.dot(z.ravel(), q.ravel()))
        x += alpha * z
        r -= alpha * q
        rr_new = float(np.dot(r.ravel(), r.ravel()))
        z = r + (rr_new / rr) * z
        rr = rr_new
    rtrue = b - np.where(S, op.apply(x), 0.0)
    return x, it, math.sqrt(float(np.dot(rtrue.ravel(), rtrue.ravel()))) / bn


def contact_boundary(S):
    """Cells of S with a 4-neighbour outside S; grid-edge cells count."""
    pad = np.pad(S, 1, constant_values=False)
    inner = pad[:-2, 1:-1] & pad[2:, 1:-1] & pad[1:-1, :-2] & pad[1:-1, 2:]
    return S & ~inner


@dataclass
class AdhesiveState:
    S: np.ndarray
    p: np.ndarray


def adhesive_step(op: Operator, f, d, state: AdhesiveState, sigma_c,
                  attach_tol, tol=1e-10, max_rounds=10000):
    """One displacement step of the adhesive procedure (Sec. 2, Eq. 12).

    Attach penetrating cells, then repeat {solve on S; detach boundary
    cells with p < -sigma_c; attach cells outside S with g < -attach_tol}
    until nothing changes.  Returns (state, rounds, u, converged).
    """
    f = np.asarray(f, dtype=np.float64)
    S = state.S.copy()
    p = np.where(S, state.p, 0.0)
    u = op.apply(p)
    S |= (f - d + u) < 0.0
    detached = np.zeros_like(S)
    rounds = 0
    converged = False
    while rounds < max_rounds:
        rounds += 1
        p, _, _ = solve_on_set(op, f, d, S, p0=p, tol=tol)
        u = op.apply(p)
        g = f - d + u
        Q = contact_boundary(S) & (p < -sigma_c)
        P = (~S) & (g < -attach_tol) & ~detached
        if not Q.any() and not P.any():
            converged = True
            break
        S = (S | P) & ~Q
        detached |= Q
        p = np.where(S, p, 0.0)
    return AdhesiveState(S, p), rounds, u, converged


def adhesive_solve(op: Operator, f, d, sigma_c, attach_tol, tol=1e-10):
    """Single adhesive solve without history: start from {f <= d}."""
    f = np.asarray(f, dtype=np.float64)
    S0 = (f - d) <= 0.0
    st = AdhesiveState(S0, np.zeros_like(f))
    return adhesive_step(op, f, d, st, sigma_c, attach_tol, tol=tol)


def sweep(op: Operator, f, d_steps, sigma_c, attach_tol, dgamma, tol=1e-10,
          state=None):
    """Quasi-static displacement-controlled sweep (Sec. 2 last paragraph).

    Carries (S, p) from step to step.  Per step records
    F = D^2 sum p, A = D^2 |S|, U_el = 1/2 D^2 sum p u, U_ad = -dgamma A.
    """
    f = np.asarray(f, dtype=np.float64)
    dA = op.dx ** 2
    if state is None:
        state = AdhesiveState(np.zeros(f.shape, dtype=bool), np.zeros_like(f))
    out = []
    for d in d_steps:
        state, rounds, u, conv = adhesive_step(op, f, d, state, sigma_c,
                                               attach_tol, tol=tol)
        A = dA * float(state.S.sum())
        out.append(dict(d=float(d), F=dA * float(state.p.sum()), area=A,
                        U_el=0.5 * dA * float(np.sum(state.p * u)),
                        U_ad=-dgamma * A, rounds=rounds, converged=conv))
    return out, state


def solve_nnls_force_singular(op, f, F, shift=None):
    """Brute-force force control for an operator whose K is only positive
    semi-definite along the uniform field (the periodic operator without a
    DC term, Eq. 11): on the constraint set D^2 sum p = F the energy
    1/2 p.K p - p.(d - f) changes by the constant c (sum p)^2 / 2 if K is
    replaced by the definite K + c 1 1^T, so that problem is solved by
    NNLS on its Cholesky factor with the approach d' bisected to the force,
    and d = d' - c sum p.  Tiny grids only."""
    dA = op.dx ** 2
    f = np.asarray(f, dtype=np.float64)
    K = op.dense_matrix()
    n = K.shape[0]
    c = float(np.trace(K)) / n if shift is None else float(shift)
    R = scipy.linalg.cholesky(K + c * np.ones((n, n)), lower=False)

    def solve(dp):
        b = scipy.linalg.solve_triangular(R, (dp - f).ravel(), trans="T", lower=False)
        p, _ = scipy.optimize.nnls(R, b, maxiter=50 * n)
        return p.reshape(f.shape)

    S = F / dA
    lo = float(f.min())
    hi = lo + 1e-3 * op.L
    while solve(hi).sum() < S:
        hi = lo + 2.0 * (hi - lo)
    dp = scipy.optimize.brentq(lambda x: solve(x).sum() - S, lo, hi, xtol=1e-15 * op.L, rtol=1e-15)
    p = solve(dp)
    return p, dp - c * float(p.sum())


@dataclass
class RetractionResult:
    state: AdhesiveState
    d: float
    F: float
    reached: bool
    steps: list
    before: AdhesiveState = None   # state of the last step above F (None if not reached)
    d_before: float = 0.0


def adhesive_force_retraction(op: Operator, f, F, d_pre, sigma_c, attach_tol, tol=1e-10,
                              steps_per_depth=32, max_steps=4096, ftol=1e-6):
    """Force-controlled retraction of an adhesive contact to a force F <= 0
    (Sec. 2 last paragraph, Eq. 12; Sec. 3.1, Eq. 19 for the instability).

    Preload: the single adhesive solve at the approach d_pre (overlap, then
    Eq. 12 rounds).  Retraction: the quasi-static displacement steps of the
    paper, d_k = d_pre - k (d_pre - min f) / steps_per_depth, each carrying
    (S, p) from the step before.  As long as the force keeps falling these
    are the equilibria a force-controlled unloading passes through; the
    first step whose force is at or below F brackets the target, and the
    approach in (d_k, d_{k-1}) carrying F is found by regula falsi over
    single steps from the state at d_{k-1} (to ftol of |F|, or of 1e-3 of
    the preload force when F is near zero).  If the contact is lost first,
    the lowest force met is the force-controlled pull-off (the force
    minimum of the retraction, Eq. 19 for a thin layer) and F is not
    reached.
    """
    f = np.asarray(f, dtype=np.float64)
    dA = op.dx ** 2
    dd = (d_pre - float(f.min())) / steps_per_depth
    st, _, _, _ = adhesive_solve(op, f, d_pre, sigma_c, attach_tol, tol=tol)
    d, Fc = d_pre, dA * float(st.p.sum())
    fabs_tol = ftol * max(abs(F), 1e-3 * abs(Fc))
    steps = [(d, Fc)]
    best = (Fc, d, st)
    for _ in range(max_steps):
        dn = d - dd
        sn, _, _, _ = adhesive_step(op, f, dn, st, sigma_c, attach_tol, tol=tol)
        Fn = dA * float(sn.p.sum())
        steps.append((dn, Fn))
        if Fn < best[0]:
            best = (Fn, dn, sn)
        if Fn <= F:
            lo, hi, Flo, Fhi = dn, d, Fn, Fc
            out = (sn, dn, Fn)
            side = 0
            for _ in range(200):
                if abs(out[2] - F) <= fabs_tol or hi - lo <= 1e-13 * dd:
                    break
                x = hi - (Fhi - F) * (hi - lo) / (Fhi - Flo)
                if not (lo < x < hi):
                    x = 0.5 * (lo + hi)
                sx, _, _, _ = adhesive_step(op, f, x, st, sigma_c, attach_tol, tol=tol)
                Fx = dA * float(sx.p.sum())
                if abs(Fx - F) < abs(out[2] - F):
                    out = (sx, x, Fx)
                if Fx < F:
                    if side == -1:
                        Fhi = F + 0.5 * (Fhi - F)
                    lo, Flo, side = x, Fx, -1
                else:
                    if side == 1:
                        Flo = F + 0.5 * (Flo - F)
                    hi, Fhi, side = x, Fx, 1
            return RetractionResult(out[0], out[1], out[2], True, steps, st, d)
        if not sn.S.any():
            return RetractionResult(best[2], best[1], best[0], False, steps)
        st, d, Fc = sn, dn, Fn
    return RetractionResult(best[2], best[1], best[0], False, steps)
