"""Physics pins: the oracle reproduces the paper's asymptotics (Sec. 3) and
the classical homogeneous limits (Hertz, Boussinesq, JKR).

Tolerances reflect discretisation (contact radius / cell size), the image
interaction of the 2N-padded period and the mesh dependence of the Eq. 12
criterion; each is stated next to its check.
"""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle.operator import Operator
from oracle.solvers import solve_pk, sweep
from oracle.transfer import Material, critical_stress, shape_factor
from paper_1807_01885_amd import inputs

pytestmark = pytest.mark.slow


@pytest.mark.parametrize("which", ["E1=E2", "h->0", "h->inf"])
def test_hertz_in_homogeneous_limits(which):
    """F = 4/3 E* R^1/2 d^3/2 with E* of the material the limit leaves."""
    N, L, R = 256, 1.0, 1.0
    mat = {"E1=E2": Material(0.1, 1.0, 0.3, 1.0, 0.3),
           "h->0": Material(1e-9, 5.0, 0.3, 1.0, 0.25),
           "h->inf": Material(1e6, 5.0, 0.3, 1.0, 0.25)}[which]
    Es = {"E1=E2": mat.E1s, "h->0": mat.E2s, "h->inf": mat.E1s}[which]
    op = Operator(N, L, mat)
    d = (L / 16) ** 2 / R
    r = solve_pk(op, inputs.paraboloid(N, L, R), d, tol=1e-9)
    a, F, p0 = an.hertz(R, d, Es)
    assert r.converged
    assert r.F == pytest.approx(F, rel=2e-3)            # discretisation, a/D = 16
    assert math.sqrt(r.area / math.pi) == pytest.approx(a, rel=1.5e-2)
    assert r.p.max() == pytest.approx(p0, rel=1e-2)


def test_boussinesq_flat_punch():
    """F = 2 a E* d; the edge singularity converges slowly (~1% at a/D = 64)."""
    N, L = 256, 1.0
    mat = Material(0.0, 1.0, 0.3, 1.0, 0.3)
    op = Operator(N, L, mat)
    a = L / 4
    d = 1e-3
    r = solve_pk(op, inputs.flat_punch(N, L, a), d, tol=1e-9)
    assert r.converged
    assert r.F == pytest.approx(an.flat_punch_force(a, d, mat.E1s), rel=2e-2)


def test_thin_layer_flat_punch_stiffness_eq14():
    """Soft layer on a (nearly) rigid base, a >> h: F = pi a^2 E~1 d / h."""
    N, L = 256, 1.0
    h = 0.004
    mat = Material(h, 1.0, 0.3, 1e5, 0.3)
    op = Operator(N, L, mat)
    a = 0.25                    # a / h = 62.5
    d = 1e-4
    r = solve_pk(op, inputs.flat_punch(N, L, a), d, tol=1e-9)
    k14 = an.thin_layer_stiffness(a, h, an.e_tilde(mat.E1, mat.nu1))
    assert r.converged
    # edge correction O(h/a) and the staircase boundary of the punch
    assert r.F / d == pytest.approx(k14, rel=4e-2)


def test_series_coefficients_eq24():
    """a_0, a_1 of Eq. 24 by quadrature of Eq. 25 (nu = 0.3)."""
    a0 = an.series_coefficient(0, 0.3)
    a1 = an.series_coefficient(1, 0.3)
    assert a0 == pytest.approx(1.3768541655, rel=1e-9)
    assert a1 == pytest.approx(-0.6275516614, rel=1e-9)
    # and a_0 = int_0^inf (1 - C_rigid(u)) du with C from Eq. 9-10
    mat = Material(1.0, 1.0, 0.3, 1e14, 0.3)
    u = np.linspace(0, 40, 400001)
    lam = 1.0 - shape_factor(u, mat)
    assert np.trapezoid(lam, u) == pytest.approx(a0, rel=1e-8)


def test_eq22_23_reduce_to_jkr():
    R, Es, dg, h = 1.0, 1.0, 1e-4, 1e16
    for a in (0.01, 0.05, 0.2):
        F, d = an.thick_layer_paraboloid(a, R, h, Es, dg, 1.37, -0.63)
        Fj, dj = an.jkr(a, R, Es, dg)
        assert F == pytest.approx(Fj, rel=1e-12)
        assert d == pytest.approx(dj, rel=1e-12)


def test_eq17_21_normalised_consistency():
    R, h, Et, dg = 1.0, 0.01, 3.0, 1e-3
    dc, ac, Fc = an.thin_layer_paraboloid_critical(R, h, Et, dg)
    for at in (0.6, 1.0, 1.7):
        F, d = an.thin_layer_paraboloid(at * ac, R, h, Et, dg)
        Fn, dn = an.thin_layer_normalised(at)
        assert F / abs(Fc) == pytest.approx(float(Fn), rel=1e-12)
        assert d / abs(dc) == pytest.approx(float(dn), rel=1e-12)
    # the minimum of F~(a~) is F~ = -1 at a~ = 1
    Fmin, _ = an.thin_layer_normalised(1.0)
    assert float(Fmin) == -1.0


def test_jkr_retraction_homogeneous():
    """Adhesive sweep on the homogeneous half-space: on retraction the
    force follows JKR's F(a) and the contact jumps off near the
    displacement-controlled JKR instability (Eq. 12 criterion, mesh
    dependent: ~10% at a/D ~ 10-30)."""
    N, L, R = 128, 1.0, 1.0
    mat = Material(0.0, 0.91, 0.3, 0.91, 0.3)      # E* = 1
    op = Operator(N, L, mat)
    dg = 2e-4
    sc = critical_stress(mat, dg, L / N)
    apo, Fpo, dpo = an.jkr_pulloff_displacement_control(R, mat.E1s, dg)
    dmax = 0.015
    steps = np.concatenate([np.linspace(0, dmax, 7)[1:],
                            np.linspace(dmax, 2.5 * dpo, 40)[1:]])
    out, _ = sweep(op, inputs.paraboloid(N, L, R), steps, sc, 1e-12 * L, dg,
                   tol=1e-9)
    Fs = [o["F"] for o in out]
    Fspan = max(Fs) - min(Fs)
    errs = []
    last_contact = None
    amax = max(o["area"] for o in out)
    for o in out[6:]:
        if o["area"] <= 0:
            continue
        last_contact = o
        a = math.sqrt(o["area"] / math.pi)
        # on the receding (JKR) branch: the area has started to shrink
        if o["area"] < amax and a / (L / N) >= 8:
            Fj, _ = an.jkr(a, R, mat.E1s, dg)
            errs.append(abs(o["F"] - Fj) / Fspan)
    assert len(errs) > 10 and max(errs) < 0.08
    assert out[-1]["area"] == 0.0
    # jump-off happens below the JKR instability, within the step size
    assert last_contact["d"] == pytest.approx(dpo, rel=0.35)
