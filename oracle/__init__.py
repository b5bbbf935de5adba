"""Plain FP64 CPU oracle for the coated half-space FFT-BEM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library,
its Python binding) may import, call, link or execute anything in this
package.  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it.

Paper: Li, Pohrt, Lyashenko, Popov, "Boundary Element Method for
non-adhesive and adhesive contacts of a coated elastic half-space"
(arXiv:1807.01885).  Each function cites the passage it follows.

Modules
  transfer  -- Fourier-space fundamental solution, Eq. 9-10 (raw and
               normalised), the per-wavenumber boundary-value problem of
               Eq. 5-8 with conditions (a)-(d), the DC term, the table.
  operator  -- u = K p by zero-padded FFT (Eq. 2, 11) and by direct sum
               (Eq. 1).
  solvers   -- the inverse problem (conjugate gradients, Sec. 2), brute
               force by NNLS, the adhesive detachment procedure (Eq. 12,
               Sec. 2 last paragraph), the quasi-static sweep.
  analytic  -- closed-form checks of Sec. 3 (Eq. 13-26) and the classical
               homogeneous limits (Hertz, Boussinesq, JKR).
  net_ref   -- FP64 reference forward/backward of the warm-start network.

Parity status: every function here is pinned by a test in tests/ against
the paper's closed forms, limits, brute force or an independent
derivation, except where a module header says "parity unpinned".
"""
