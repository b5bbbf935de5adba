"""GPU parity of the preconditioned constrained CG (stiff thin coatings,
where the layer-removing Fourier preconditioner is used) against the FP64
oracle's plain constrained CG.  The converged pressure is the unique
solution of the complementarity problem, so both must agree to the
solve tolerance; the preconditioned path must also need fewer iterations.
precond = 3 (two-phase; the automatic choice on stiff thin coatings) runs
the plain or layer-preconditioned iteration until an iteration leaves the
contact set unchanged, then switches to the inverse of the operator's
symbol."""
import numpy as np
import pytest
import torch

from oracle.operator import Operator
from oracle.solvers import solve_pk
from oracle.transfer import Material
from paper_1807_01885_amd import inputs

pytestmark = pytest.mark.gpu
DT = {"fp64": torch.float64, "fp32": torch.float32}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,mat,F", [
    ("cone", Material(0.011, 87.8, 0.31, 1.0, 0.33), 0.0188),
    ("flat", Material(0.0083, 34.7, 0.36, 1.0, 0.21), 3.3e-4),
    ("ellipse", Material(0.0026, 12.1, 0.3, 1.0, 0.3), 4e-3),
])
def test_preconditioned_force_solve(lib, prec, shape, mat, F):
    print(f"precond {shape} {prec}", flush=True)
    N, L = 128, 1.0
    f = {"cone": inputs.cone(N, L, 0.125), "flat": inputs.flat_punch(N, L, 0.09),
         "ellipse": inputs.elliptic_punch(N, L, 0.13, 0.06)}[shape]
    op = Operator(N, L, mat)
    ref = solve_pk(op, f, F, mode="force", tol=1e-10)
    plan = lib.cb_plan_create(N, L, mat.h, mat.E1, mat.nu1, mat.E2, mat.nu2, 0.0, prec)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-8
    out = {}
    for pc in (1, 0, 3, -1):
        p = torch.zeros_like(ft)
        res = lib.cb_solve_force(plan, ft, F, p, tol=tol, precond=pc)
        e_p = np.linalg.norm(p.double().cpu().numpy() - ref.p) / np.linalg.norm(ref.p)
        out[pc] = (res["iters"], e_p, res)
        print(f"  precond={pc:+d} iters {res['iters']} (oracle plain {ref.iters}) e_p {e_p:.2e} d {res['d']:.6e}")
        assert res["status"] == 0
        assert e_p < (1e-7 if prec == "fp64" else 2e-4)
        assert abs(res["F"] - F) / F < (1e-12 if prec == "fp64" else 1e-6)
    assert out[1][0] < out[0][0]          # fewer iterations with the preconditioner
    assert out[-1][0] == out[3][0]        # automatic choice: two-phase


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("pc", [1, 0, 3])
def test_initial_guess_with_too_small_contact(lib, prec, pc):
    """An initial guess whose support is smaller than the contact (the
    oracle's pressure with its low-pressure rim removed) makes the solver
    grow the contact set; activated cells take a step scaled to the
    search direction, so the preconditioned solve converges to the same
    pressure as the plain one and the oracle."""
    print(f"grow contact pc={pc} {prec}", flush=True)
    N, L = 128, 1.0
    mat = Material(0.0023, 42.8, 0.31, 1.0, 0.30)
    f = inputs.cone(N, L, 0.116)
    F = 5.6e-3
    op = Operator(N, L, mat)
    ref = solve_pk(op, f, F, mode="force", tol=1e-10)
    # keep the inner 70% of the contact radius, with a 20% ripple
    a = np.sqrt((ref.p > 0).sum() / np.pi) * (L / N)
    yy, xx = (np.indices((N, N)) - N // 2) * (L / N)
    p0 = np.where(np.hypot(xx, yy) < 0.7 * a, ref.p, 0.0)
    p0 = np.ascontiguousarray(p0 * (1.0 + 0.2 * np.cos(np.arange(N) * 0.3))[None, :])
    assert (p0 > 0).sum() < 0.6 * (ref.p > 0).sum()
    plan = lib.cb_plan_create(N, L, mat.h, mat.E1, mat.nu1, mat.E2, mat.nu2, 0.0, prec)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    p = torch.tensor(p0, dtype=torch.float64, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-8
    res = lib.cb_solve_force(plan, ft, F, p, tol=tol, precond=pc, init=1, max_iter=4000)
    e_p = np.linalg.norm(p.cpu().numpy() - ref.p) / np.linalg.norm(ref.p)
    print(f"  iters {res['iters']} (oracle cold {ref.iters}) e_p {e_p:.2e}", flush=True)
    assert res["status"] == 0
    assert e_p < (1e-7 if prec == "fp64" else 2e-4)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,mat,F", [
    ("paraboloid", Material(0.08, 0.3, 0.3, 1.0, 0.3), 1.5e-3),
    ("flat", Material(0.02, 1.0, 0.25, 1.0, 0.35), 4e-4),
    ("ellipse", Material(0.2, 20.0, 0.3, 1.0, 0.3), 3e-3),
])
def test_inverse_symbol_preconditioner(lib, prec, shape, mat, F):
    """precond = 2 (the inverse of the operator's symbol, the automatic
    choice from a caller's guess): same pressure as the oracle's plain
    method, fewer iterations than the plain GPU method; on these coatings
    the automatic choice from the estimated force start is the inverse
    symbol throughout."""
    print(f"inverse precond {shape} {prec}", flush=True)
    N, L = 128, 1.0
    f = {"paraboloid": inputs.paraboloid(N, L, 1.0), "flat": inputs.flat_punch(N, L, 0.11),
         "ellipse": inputs.elliptic_punch(N, L, 0.14, 0.07)}[shape]
    ref = solve_pk(Operator(N, L, mat), f, F, mode="force", tol=1e-10)
    plan = lib.cb_plan_create(N, L, mat.h, mat.E1, mat.nu1, mat.E2, mat.nu2, 0.0, prec)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-8
    it = {}
    for pc in (2, 0, 3, -1):
        p = torch.zeros_like(ft)
        res = lib.cb_solve_force(plan, ft, F, p, tol=tol, precond=pc)
        e_p = np.linalg.norm(p.cpu().numpy() - ref.p) / np.linalg.norm(ref.p)
        print(f"  precond={pc:+d} iters {res['iters']} (oracle plain {ref.iters}) e_p {e_p:.2e}", flush=True)
        assert res["status"] == 0
        assert e_p < (1e-7 if prec == "fp64" else 2e-4)
        it[pc] = res["iters"]
    assert it[2] < it[0] and it[-1] == it[2]
    with pytest.raises(lib.CoatbemError):
        lib.cb_solve_force(plan, ft, F, torch.zeros_like(ft), precond=4)
