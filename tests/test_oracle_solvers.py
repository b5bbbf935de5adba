"""Pins of the oracle's inverse problems (Sec. 2 after Eq. 11; Eq. 12).

The conjugate-gradient contact solve is pinned to brute force (NNLS on the
Cholesky factor of the dense K, whose KKT conditions are the contact
complementarity problem), its KKT residuals, and the fixed-set solve to a
dense linear solve.  The adhesive bookkeeping (boundary set) is pinned on
hand-built masks.
"""
import math

import numpy as np
import pytest

from oracle.operator import Operator
from oracle.solvers import (AdhesiveState, adhesive_step, contact_boundary,
                            self_influence, solve_nnls, solve_nnls_force,
                            solve_on_set, solve_pk, sweep)
from oracle.transfer import Material
from paper_1807_01885_amd import inputs

LAYER = Material(0.1, 10.0, 0.3, 1.0, 0.3)
SOFT = Material(0.05, 0.2, 0.3, 1.0, 0.3)


def _kkt(op, f, d, p):
    g = op.apply(p) + f - d
    on = p > 0
    return (float(np.abs(g[on]).max() / abs(d - f.min())) if on.any() else 0.0,
            float(max(0.0, -g[~on].min()) / abs(d - f.min())) if (~on).any() else 0.0)


@pytest.mark.parametrize("mat", [LAYER, SOFT])
@pytest.mark.parametrize("shape", ["paraboloid", "cone", "flat"])
def test_pk_equals_nnls_brute_force(mat, shape):
    N, L = 16, 1.0
    op = Operator(N, L, mat)
    f = {"paraboloid": inputs.paraboloid(N, L, 1.0),
         "cone": inputs.cone(N, L, 0.1),
         "flat": inputs.flat_punch(N, L, 0.2)}[shape]
    d = {"paraboloid": 0.01, "cone": 0.02, "flat": 1e-3}[shape]
    r = solve_pk(op, f, d, tol=1e-12)
    assert r.converged
    pn = solve_nnls(op, f, d)
    assert np.array_equal(r.p > 0, pn > 0)
    np.testing.assert_allclose(r.p, pn, rtol=0, atol=1e-9 * pn.max())
    on_res, off_res = _kkt(op, f, d, r.p)
    assert on_res < 1e-10 and off_res < 1e-10


def test_pk_force_control_equals_brute_force():
    N, L = 16, 1.0
    op = Operator(N, L, SOFT)
    f = inputs.paraboloid(N, L, 1.0)
    F = 3e-5
    r = solve_pk(op, f, F, mode="force", tol=1e-12)
    assert r.converged
    assert r.F == pytest.approx(F, rel=1e-12)
    pn, dn = solve_nnls_force(op, f, F)
    assert r.d == pytest.approx(dn, rel=1e-8)
    np.testing.assert_allclose(r.p, pn, rtol=0, atol=1e-7 * pn.max())


def test_config1_brute_force():
    """N = 64 paraboloid on the h = 0.1, E1/E2 = 10 coating: residual
    1e-10 and the brute-force pressure."""
    c = inputs.paraboloid_c1()
    op = Operator(c.N, c.L, Material(c.h, c.E1, c.nu1, c.E2, c.nu2))
    r = solve_pk(op, c.f, c.target, tol=1e-10)
    assert r.converged and r.resid <= 1e-10
    pn = solve_nnls(op, c.f, c.target)
    assert np.linalg.norm(r.p - pn) / np.linalg.norm(pn) < 1e-8
    assert np.array_equal(r.p > 0, pn > 0)


def test_no_overlap_gives_zero():
    op = Operator(16, 1.0, LAYER)
    f = inputs.paraboloid(16, 1.0, 1.0)
    r = solve_pk(op, f, -1e-3)
    assert r.converged and not r.p.any()


def test_solve_on_set_equals_dense_solve():
    N, L = 12, 1.0
    op = Operator(N, L, SOFT)
    f = inputs.paraboloid(N, L, 1.0)
    S = f <= 0.02
    d = 0.005
    p, it, res = solve_on_set(op, f, d, S, tol=1e-13)
    K = op.dense_matrix()
    idx = np.flatnonzero(S.ravel())
    ps = np.linalg.solve(K[np.ix_(idx, idx)], (d - f.ravel())[idx])
    ref = np.zeros(N * N)
    ref[idx] = ps
    np.testing.assert_allclose(p.ravel(), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    assert (p.ravel()[idx] < 0).any()  # tension appears: adhesive solve is unconstrained
    assert res < 1e-12


def test_contact_boundary_masks():
    S = np.zeros((6, 6), dtype=bool)
    S[1:5, 1:5] = True
    B = contact_boundary(S)
    expect = S.copy()
    expect[2:4, 2:4] = False
    assert np.array_equal(B, expect)
    full = np.ones((4, 4), dtype=bool)
    Bf = contact_boundary(full)          # grid-edge cells are boundary
    exp = np.ones((4, 4), dtype=bool)
    exp[1:3, 1:3] = False
    assert np.array_equal(Bf, exp)
    single = np.zeros((5, 5), dtype=bool)
    single[2, 2] = True
    assert np.array_equal(contact_boundary(single), single)


def test_adhesive_step_zero_adhesion_is_nonadhesive_limit():
    """sigma_c -> 0 with no tension allowed reduces to the complementarity
    solution only if every tensile boundary cell peels; with sigma_c = inf
    nothing detaches and the fixed-set solve is returned."""
    N, L = 16, 1.0
    op = Operator(N, L, SOFT)
    f = inputs.paraboloid(N, L, 1.0)
    d = 0.004
    st = AdhesiveState(f <= d, np.zeros_like(f))
    st2, rounds, u, conv = adhesive_step(op, f, d, st, math.inf, 1e-12)
    p_set, _, _ = solve_on_set(op, f, d, st.S, tol=1e-10)
    assert conv
    # with sigma_c infinite the contact only grows by penetration
    assert (st2.S >= st.S).all()
    st3, _, _, conv3 = adhesive_step(op, f, d, st, 0.0, 1e-12)
    r = solve_pk(op, f, d, tol=1e-12)
    assert conv3
    # peeling every tensile boundary cell leaves a compressive contact
    assert st3.p[st3.S].min() > -1e-9 * r.p.max()
    assert abs(st3.p.sum() - r.p.sum()) < 1e-3 * r.p.sum()


def test_sweep_records_energy_terms():
    N, L = 16, 1.0
    op = Operator(N, L, SOFT)
    f = inputs.paraboloid(N, L, 1.0)
    out, st = sweep(op, f, [0.002, 0.004], 1.0, 1e-12, 1e-4)
    for o in out:
        assert o["U_ad"] == pytest.approx(-1e-4 * o["area"])
        assert o["U_el"] > 0 and o["F"] > 0
