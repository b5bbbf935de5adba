"""Seeded synthetic inputs (indenter profiles and workload recipes).

This module holds no arithmetic of the contact method: it only draws the
geometry and material parameters that both the GPU library and the CPU
checker are fed.  Everything is deterministic given its seed.

Grid convention (Sec. 2, Fig. 2 of the paper): N x N square cells of size
Delta = L/N, row index i (y), column index j (x); the centre of cell (i, j)
is ((j - N/2) Delta, (i - N/2) Delta), so a centred apex sits on cell
(N/2, N/2).  Profiles f >= 0 with min f = 0 at the apex.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SHAPES = ("paraboloid", "cone", "flat", "ellipse")


def coords(N, L):
    dx = L / N
    x = (np.arange(N) - N // 2) * dx
    return np.meshgrid(x, x, indexing="xy")  # X[i, j] = x_j, Y[i, j] = y_i


def paraboloid(N, L, R):
    X, Y = coords(N, L)
    return (X * X + Y * Y) / (2.0 * R)


def cone(N, L, tan_beta):
    X, Y = coords(N, L)
    return np.sqrt(X * X + Y * Y) * tan_beta


def flat_punch(N, L, a, big=None):
    """Flat-ended cylinder of radius a; outside the face the profile is
    `big` (default L), far beyond any approach used."""
    X, Y = coords(N, L)
    big = L if big is None else big
    return np.where(X * X + Y * Y <= a * a, 0.0, big)


def elliptic_punch(N, L, ax, ay, big=None):
    X, Y = coords(N, L)
    big = L if big is None else big
    return np.where((X / ax) ** 2 + (Y / ay) ** 2 <= 1.0, 0.0, big)


def rough_surface(N, L, hurst=0.7, qr_factor=4.0, rms=None, seed=0):
    """Gaussian isotropic self-affine surface by random phases.

    Power spectrum C(q) = C0 for 2 pi/L <= q < q_r, C0 (q/q_r)^(-2(1+H))
    for q_r <= q <= q_s, zero elsewhere; q_r = qr_factor * 2 pi/L,
    q_s = pi/Delta.  Scaled to the given rms height (default 1e-3 L).
    Returned as an indenter profile f = max(z) - z >= 0.
    """
    rng = np.random.default_rng(seed)
    dx = L / N
    q1 = 2.0 * np.pi * np.fft.fftfreq(N, d=dx)
    q0 = 2.0 * np.pi * np.fft.rfftfreq(N, d=dx)
    q = np.sqrt(q1[:, None] ** 2 + q0[None, :] ** 2)
    qL = 2.0 * np.pi / L
    qr = qr_factor * qL
    qs = np.pi / dx
    C = np.where(q < qr, 1.0, (np.maximum(q, qr) / qr) ** (-2.0 * (1.0 + hurst)))
    C = np.where((q >= qL * (1 - 1e-12)) & (q <= qs * (1 + 1e-12)), C, 0.0)
    amp = np.sqrt(C) * (rng.standard_normal(q.shape) + 1j * rng.standard_normal(q.shape))
    z = np.fft.irfft2(amp, s=(N, N))
    z -= z.mean()
    target = 1e-3 * L if rms is None else rms
    z *= target / z.std()
    return z.max() - z


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------
@dataclass
class Case:
    """One contact problem: grid, material, indenter, load."""

    N: int
    L: float
    h: float
    E1: float
    nu1: float
    E2: float
    nu2: float
    dgamma: float
    shape: str
    f: np.ndarray = field(repr=False)
    mode: str            # "disp" (target = d) or "force" (target = F)
    target: float
    meta: dict = field(default_factory=dict)


def paraboloid_c1():
    """Non-adhesive paraboloid, N = 64, L = 4, h = 0.1, E1 = 10, E2 = 1,
    nu = 0.3, R = 1, d = 0.01 (FP64, residual 1e-10)."""
    N, L = 64, 4.0
    return Case(N, L, 0.1, 10.0, 0.3, 1.0, 0.3, 0.0, "paraboloid",
                paraboloid(N, L, 1.0), "disp", 0.01, dict(R=1.0))


def adhesive_sweep_c2():
    """Six adhesive paraboloid sweeps at N = 512, L = 2, R = 1,
    dgamma = 1e-3 E2 R, h in {0.02, 0.1, 0.5}, E1/E2 in {0.1, 10}.

    Each sweep: 80 approach steps 0 -> (L/8)^2/R, then 120 retraction
    steps down to -2 |d_c| with the homogeneous JKR estimate
    |d_c| = 3/4 (pi^2 dgamma^2 R / E1*^2)^(1/3) of the coating.
    """
    N, L, R, E2, nu = 512, 2.0, 1.0, 1.0, 0.3
    dgamma = 1e-3 * E2 * R
    out = []
    for h in (0.02, 0.1, 0.5):
        for E1 in (0.1, 10.0):
            E1s = E1 / (1 - nu * nu)
            dmax = (L / 8.0) ** 2 / R
            dc = 0.75 * (math.pi ** 2 * dgamma ** 2 * R / E1s ** 2) ** (1.0 / 3.0)
            steps = np.concatenate([np.linspace(0.0, dmax, 81)[1:],
                                    np.linspace(dmax, -2.0 * dc, 121)[1:]])
            out.append(Case(N, L, h, E1, nu, E2, nu, dgamma, "paraboloid",
                            paraboloid(N, L, R), "sweep", 0.0,
                            dict(R=R, d_steps=steps)))
    return out


def flat_and_rough_c3(N=2048, seeds=(0, 1, 2)):
    """Flat punch (a = 0.5) and rough indenters on h = 0.05, E1/E2 = 0.05,
    L = 2, nu = 0.3; d = 2e-3 for the punch, 2 x rms past first touch
    for the rough surfaces."""
    L, h, E1, E2, nu = 2.0, 0.05, 0.05, 1.0, 0.3
    out = [Case(N, L, h, E1, nu, E2, nu, 0.0, "flat", flat_punch(N, L, 0.5),
                "disp", 2e-3, dict(a=0.5))]
    for s in seeds:
        f = rough_surface(N, L, seed=s)
        out.append(Case(N, L, h, E1, nu, E2, nu, 0.0, "rough", f, "disp",
                        2.0 * 1e-3 * L, dict(seed=s)))
    return out


def _loguniform(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def batch_c4(n=256, seed=4, N_choices=(128, 256, 512, 1024), L=1.0,
             adhesion=True):
    """Batched workload: uneven grids, four indenter families, random
    coatings, half of the cases adhesive.

    N uniform in N_choices; shape uniform over paraboloid (R = 1), cone
    (tan beta ~ U[0.02, 0.2]), flat punch, elliptic punch (aspect
    ~ U[1, 4]); overlap radius r ~ U[L/16, L/6] sets d (punches: a = r,
    d ~ logU[1e-4, 1e-2] L); h/L ~ logU[1e-3, 0.3]; E2 = 1,
    E1/E2 ~ logU[0.01, 100]; nu1, nu2 ~ U[0.2, 0.45].  Adhesive cases
    (dgamma = w E2* L, w ~ logU[1e-5, 1e-3]) are single displacement-
    controlled solves.  Non-adhesive cases are force-controlled with the
    load of the homogeneous closed form at that d, evaluated with the
    geometric-mean modulus sqrt(E1* E2*) (a load of the right order; the
    contact radius it produces is not r).
    """
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(n):
        N = int(rng.choice(N_choices))
        shape = SHAPES[int(rng.integers(0, 4))]
        r = rng.uniform(L / 16.0, L / 6.0)
        h = _loguniform(rng, 1e-3, 0.3) * L
        E2 = 1.0
        E1 = _loguniform(rng, 0.01, 100.0) * E2
        nu1 = float(rng.uniform(0.2, 0.45))
        nu2 = float(rng.uniform(0.2, 0.45))
        adh = bool(adhesion and rng.uniform() < 0.5)
        w = _loguniform(rng, 1e-5, 1e-3)
        tanb = float(rng.uniform(0.02, 0.2))
        aspect = float(rng.uniform(1.0, 4.0))
        dpunch = _loguniform(rng, 1e-4, 1e-2) * L
        meta = dict(r=r)
        if shape == "paraboloid":
            R = 1.0
            f = paraboloid(N, L, R)
            d = r * r / (2.0 * R)
            meta["R"] = R
        elif shape == "cone":
            f = cone(N, L, tanb)
            d = r * tanb
            meta["tan_beta"] = tanb
        elif shape == "flat":
            f = flat_punch(N, L, r)
            d = dpunch
            meta["a"] = r
        else:
            f = elliptic_punch(N, L, r, r / aspect)
            d = dpunch
            meta["a"] = r
            meta["aspect"] = aspect
        E1s = E1 / (1 - nu1 * nu1)
        E2s = E2 / (1 - nu2 * nu2)
        Es = math.sqrt(E1s * E2s)
        if adh:
            dgamma = w * E2s * L
            cases.append(Case(N, L, h, E1, nu1, E2, nu2, dgamma, shape, f,
                              "disp", d, meta))
        else:
            if shape == "paraboloid":
                F = 4.0 / 3.0 * Es * math.sqrt(meta["R"]) * d ** 1.5
            elif shape == "cone":
                F = 2.0 / math.pi * Es * d * d / tanb
            elif shape == "flat":
                F = 2.0 * r * Es * d
            else:
                F = 2.0 * r * math.sqrt(1.0 / aspect) * Es * d
            cases.append(Case(N, L, h, E1, nu1, E2, nu2, 0.0, shape, f,
                              "force", F, meta))
    return cases


def headline_set(n=32, seed=1024, N=1024):
    """The N = 1024 solve set: the batched recipe with the grid fixed and
    adhesion off (force-controlled solves, the learned warm start's
    input form)."""
    return batch_c4(n=n, seed=seed, N_choices=(N,), adhesion=False)
