"""GPU parity of the preconditioned constrained CG (stiff thin coatings,
where the layer-removing Fourier preconditioner is used) against the FP64
oracle's plain constrained CG.  The converged pressure is the unique
solution of the complementarity problem, so both must agree to the
solve tolerance; the preconditioned path must also need fewer iterations."""
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
    for pc in (1, 0, -1):
        p = torch.zeros_like(ft)
        res = lib.cb_solve_force(plan, ft, F, p, tol=tol, precond=pc)
        e_p = np.linalg.norm(p.double().cpu().numpy() - ref.p) / np.linalg.norm(ref.p)
        out[pc] = (res["iters"], e_p, res)
        print(f"  precond={pc:+d} iters {res['iters']} (oracle plain {ref.iters}) e_p {e_p:.2e} d {res['d']:.6e}")
        assert res["status"] == 0
        assert e_p < (1e-7 if prec == "fp64" else 2e-4)
        assert abs(res["F"] - F) / F < (1e-12 if prec == "fp64" else 1e-6)
    assert out[1][0] < out[0][0]          # fewer iterations with the preconditioner
    assert out[-1][0] == out[1][0]        # automatic choice turns it on here
