"""Closed-form contact solutions used to pin the oracle (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Eq. 4: homogeneous transfer function (limit check of Eq. 9).
  * Eq. 12: mesh-dependent critical stress.
  * Eq. 13: critical separation from the non-adhesive incremental
    stiffness k(a) of an axisymmetric contact.
  * Eq. 14-16: soft layer on a rigid base, flat punch, a >> h.
  * Eq. 17-21: soft layer on a rigid base, paraboloid, a >> h.
  * Eq. 22-25: thick layer, paraboloid, eps = a/h << 1, coefficients a_m
    from Lambda(u) with L = 4 nu - 3 (not the domain size).
  * Eq. 26: adhesion parameter alpha.
Classical homogeneous solutions (textbook, e.g. Johnson, Contact
Mechanics): Hertz, Boussinesq flat punch, uniformly loaded disc, JKR.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate


def reduced_modulus(E, nu):
    """E* = E / (1 - nu^2), Eq. 4."""
    return E / (1.0 - nu * nu)


# ---------------------------------------------------------------------------
# Homogeneous half-space (limits h -> 0, h -> inf, E1 = E2)
# ---------------------------------------------------------------------------
def hertz(R, d, Es):
    """Hertz: a = sqrt(R d), F = 4/3 E* R^1/2 d^3/2, p0 = 2 E* a/(pi R)."""
    a = math.sqrt(R * d)
    F = 4.0 / 3.0 * Es * math.sqrt(R) * d ** 1.5
    p0 = 2.0 * Es * a / (math.pi * R)
    return a, F, p0


def hertz_pressure(r, a, p0):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < a, p0 * np.sqrt(np.clip(1.0 - (r / a) ** 2, 0, None)), 0.0)


def hertz_pressure_displacement(r, a, p0, Es):
    """Surface displacement under the Hertz pressure, r <= a:
    u = pi p0 (2 a^2 - r^2) / (4 a E*)."""
    r = np.asarray(r, dtype=np.float64)
    return math.pi * p0 * (2 * a * a - r * r) / (4.0 * a * Es)


def flat_punch_force(a, d, Es):
    """Boussinesq flat punch: F = 2 a E* d."""
    return 2.0 * a * Es * d


def uniform_disc_displacement(p0, a, Es):
    """Uniform pressure p0 on a disc of radius a: u(0) = 2 p0 a / E*,
    u(a) = 4 p0 a / (pi E*)."""
    return 2.0 * p0 * a / Es, 4.0 * p0 * a / (math.pi * Es)


def jkr(a, R, Es, dgamma):
    """JKR: F = 4 E* a^3/(3R) - sqrt(8 pi dgamma E* a^3),
    d = a^2/R - sqrt(2 pi dgamma a / E*)."""
    F = 4.0 * Es * a ** 3 / (3.0 * R) - math.sqrt(8.0 * math.pi * dgamma * Es * a ** 3)
    d = a * a / R - math.sqrt(2.0 * math.pi * dgamma * a / Es)
    return F, d


def jkr_pulloff_displacement_control(R, Es, dgamma):
    """Displacement-controlled JKR instability: dd/da = 0,
    a^3 = pi dgamma R^2 / (8 E*)."""
    a = (math.pi * dgamma * R * R / (8.0 * Es)) ** (1.0 / 3.0)
    F, d = jkr(a, R, Es, dgamma)
    return a, F, d


# ---------------------------------------------------------------------------
# Eq. 12-21: critical stress, thin layer on a rigid base
# ---------------------------------------------------------------------------
def critical_stress(E1s, dgamma, dx):
    """Eq. 12."""
    return math.sqrt(E1s * dgamma / (0.473201 * dx))


def e_tilde(E1, nu1):
    """Eq. 15: E~1 = E1 (1 - nu1) / ((1 + nu1)(1 - 2 nu1))."""
    return E1 * (1.0 - nu1) / ((1.0 + nu1) * (1.0 - 2.0 * nu1))


def thin_layer_stiffness(a, h, Et):
    """Eq. 14: k = pi a^2 E~1 / h."""
    return math.pi * a * a * Et / h


def thin_layer_flat_punch_critical(a, h, Et, dgamma):
    """Eq. 16: d_c = -sqrt(2 dgamma h / E~1), F_c = k d_c."""
    dc = -math.sqrt(2.0 * dgamma * h / Et)
    Fc = -math.pi * a * a * math.sqrt(2.0 * Et * dgamma / h)
    return dc, Fc


def critical_separation_eq13(dk_da, a, dgamma):
    """Eq. 13 solved for |d_c|: dk/da * d_c^2 / 2 = 2 pi a dgamma."""
    return math.sqrt(4.0 * math.pi * a * dgamma / dk_da)


def thin_layer_paraboloid(a, R, h, Et, dgamma):
    """Eq. 17-18: F(a), d(a) for a paraboloid on a thin layer, a >> h."""
    s = math.sqrt(2.0 * h * dgamma / Et)
    F = math.pi * Et * a * a / h * (a * a / (4.0 * R) - s)
    d = a * a / (2.0 * R) - s
    return F, d


def thin_layer_paraboloid_critical(R, h, Et, dgamma):
    """Eq. 19: d_crit, a_crit, F_crit."""
    dcrit = -math.sqrt(2.0 * h * dgamma / Et)
    acrit = (8.0 * R * R * h * dgamma / Et) ** 0.25
    Fcrit = -2.0 * math.pi * R * dgamma
    return dcrit, acrit, Fcrit


def thin_layer_normalised(at):
    """Eq. 20-21: F~ = a~^4 - 2 a~^2, d~ = a~^2 - 1."""
    at = np.asarray(at, dtype=np.float64)
    return at ** 4 - 2.0 * at ** 2, at ** 2 - 1.0


# ---------------------------------------------------------------------------
# Eq. 22-26: thick layer series
# ---------------------------------------------------------------------------
def Lambda(u, nu):
    """Eq. 25 with L = 4 nu - 3."""
    L = 4.0 * nu - 3.0
    u = np.asarray(u, dtype=np.float64)
    e2 = np.exp(-2.0 * u)
    e4 = e2 * e2
    num = 2.0 * L * e4 - (L * L + 1.0 + 4.0 * u + 4.0 * u * u) * e2
    den = L - (L * L + 1.0 + 4.0 * u * u) * e2 + L * e4
    return num / den


def series_coefficient(m, nu):
    """Eq. 24: a_m = (-1)^m / (2^{2m} (m!)^2) int_0^inf Lambda(u) u^{2m} du."""
    val, _ = scipy.integrate.quad(lambda u: float(Lambda(u, nu)) * u ** (2 * m),
                                  0.0, np.inf, limit=400, epsabs=0.0,
                                  epsrel=1e-13)
    return (-1.0) ** m / (2.0 ** (2 * m) * math.factorial(m) ** 2) * val


def thick_layer_paraboloid(a, R, h, E1s, dgamma, a0, a1):
    """Eq. 22-23: F(a), d(a) for eps = a/h << 1."""
    eps = a / h
    pi = math.pi
    s = math.sqrt(2.0 * pi * E1s * a * dgamma)
    F = (4.0 * E1s * a ** 3 / (3.0 * R) * (1.0 - eps ** 3 * 8.0 * a1 / (3.0 * pi))
         * (1.0 - 3.0 * R * s / (2.0 * E1s * a * a)))
    d = a * a / R * (1.0 - eps * 4.0 * a0 / (3.0 * pi) - eps ** 3 * 16.0 * a1 / (5.0 * pi)
                     + eps ** 4 * 32.0 * a0 * a1 / (9.0 * pi * pi)
                     - R * s / (E1s * a * a) * (1.0 - eps * 2.0 * a0 / pi
                                                - eps ** 3 * 16.0 * a1 / (3.0 * pi)
                                                + eps ** 4 * 16.0 * a0 * a1 / (3.0 * pi * pi)))
    return F, d


def adhesion_parameter(dgamma, R, E1s, h):
    """Eq. 26: alpha = sqrt(2 dgamma R^2 / (E1* h^3))."""
    return math.sqrt(2.0 * dgamma * R * R / (E1s * h ** 3))
