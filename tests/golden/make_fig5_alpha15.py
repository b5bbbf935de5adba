"""Write tests/golden/fig5_alpha15_d8.json: the FP64 oracle's quasi-static
adhesive sweep (Sec. 2 last paragraph, Eq. 12) of the paper's large-alpha
case of Fig. 5: a paraboloid with alpha = 15 (Eq. 26) on a thin layer on a
rigid base (E2 = 1e5 E1, nu = 0.3, dgamma = 1e-3 E1* h), cells D = h/8,
N = 256; approach to 1.25 |d_crit| (Eq. 19) in 8 steps, retraction to
-1.3 |d_crit| in 60 steps.

Per step: d, F = D^2 sum p, area D^2 |S|, U_el = 1/2 D^2 sum p u, the
detach/attach rounds and a hash of the contact set (sha256 of its packed
bits, 16 hex digits).  Calls only oracle/ and the seeded input recipe,
which holds no arithmetic of the method.  Offline (about a minute):
    python tests/golden/make_fig5_alpha15.py
"""
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import analytic as an  # noqa: E402
from oracle.operator import Operator  # noqa: E402
from oracle.solvers import AdhesiveState, adhesive_step  # noqa: E402
from oracle.transfer import Material, critical_stress  # noqa: E402
from paper_1807_01885_amd import inputs  # noqa: E402

TOL = 1e-10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig5_alpha15_d8.json")
H, N, CELLS_PER_H, ALPHA = 1.0, 256, 8, 15.0


def mask_hash(S):
    return hashlib.sha256(np.packbits(S.astype(bool)).tobytes()).hexdigest()[:16]


def setup():
    """Material, grid, R and the displacement steps of the sweep."""
    D = H / CELLS_PER_H
    L = N * D
    mat = Material(H, 1.0, 0.3, 1e5, 0.3)
    Et = an.e_tilde(mat.E1, mat.nu1)
    dg = 1e-3 * mat.E1s * H
    R = ALPHA * math.sqrt(mat.E1s * H ** 3 / (2.0 * dg))
    dcr, acr, Fcr = an.thin_layer_paraboloid_critical(R, H, Et, dg)
    dmax = 1.25 * abs(dcr)
    steps = np.concatenate([np.linspace(0, dmax, 9)[1:], np.linspace(dmax, -1.3 * abs(dcr), 61)[1:]])
    return mat, D, L, dg, R, steps


def main():
    mat, D, L, dg, R, steps = setup()
    op = Operator(N, L, mat)
    sc = critical_stress(mat, dg, D)
    atol = 1e-12 * L
    f = inputs.paraboloid(N, L, R)
    dA = D * D
    st = AdhesiveState(np.zeros((N, N), dtype=bool), np.zeros((N, N)))
    rec = []
    t0 = time.time()
    for k, d in enumerate(steps):
        st, rounds, u, conv = adhesive_step(op, f, float(d), st, sc, atol, tol=TOL)
        assert conv
        rec.append(dict(d=float(d), F=dA * float(st.p.sum()), area=dA * float(st.S.sum()),
                        U_el=0.5 * dA * float(np.sum(st.p * u)), rounds=int(rounds), mask=mask_hash(st.S)))
        print(f"step {k:3d} d={d:+.4e} F={rec[-1]['F']:+.6e} area={rec[-1]['area']:.6f} rounds={rounds} "
              f"{time.time() - t0:.0f}s", flush=True)
    out = dict(source="oracle.solvers.adhesive_step (FP64), Sec. 2 last paragraph, Eq. 12",
               case="Fig. 5, alpha = 15 (Eq. 26), thin layer on a rigid base", N=N, L=L, h=mat.h, E1=mat.E1,
               nu1=mat.nu1, E2=mat.E2, nu2=mat.nu2, dgamma=dg, R=R, sigma_c=sc, attach_tol=atol, tol=TOL,
               mask_hash="sha256 of numpy.packbits(contact set, row-major), first 16 hex digits", steps=rec)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
