/*
 * libcoatbem -- boundary element method for the frictionless normal contact
 * of a rigid indenter with an elastic layer (h, E1, nu1) bonded to an
 * elastic half-space (E2, nu2), non-adhesive and adhesive, on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Li, Pohrt, Lyashenko, Popov, "Boundary Element Method for
 * non-adhesive and adhesive contacts of a coated elastic half-space",
 * arXiv:1807.01885.  Section, equation and figure numbers below refer to it.
 *
 * Conventions shared by every entry point
 *   - Grid (Sec. 2, Fig. 2): an L x L square of N x N cells, Delta = L/N.
 *     Arrays are N*N, row-major, element (i, j) at i*N + j, row i = y,
 *     column j = x; the centre of cell (i, j) is ((j-N/2)Delta, (i-N/2)Delta).
 *   - Pressure p > 0 is compressive (sigma_zz = -p at z = 0, condition (c));
 *     u is the surface displacement into the body; f >= 0 is the indenter
 *     profile; d is the rigid approach (positive into the body); the gap is
 *     g = f - d + u; the total force is F = Delta^2 * sum(p).
 *   - cb_apply_K takes p and u in the plan's precision (double for CB_FP64,
 *     float for CB_FP32).  The solve and sweep calls take f, p and the
 *     sweep state as double for every plan: the solution state is kept in
 *     FP64, and CB_FP32 plans run the convolutions of the search directions
 *     in FP32 (see cb_plan_opts.precision).  Masks are uint8, 1 = in contact.
 *   - Every array pointer is a DEVICE pointer on the plan's device unless
 *     the name says _host.  The caller owns every array; the library never
 *     frees or retains caller memory beyond the call.  The library owns the
 *     plan, its tables and its workspace.
 *   - Work is enqueued on the plan's stream.  cb_apply_K is asynchronous.
 *     The solve and sweep calls synchronise the stream before they fill
 *     their host result structs and return.
 *   - Errors are returned as negative status codes, never thrown across
 *     the ABI; cb_last_error() gives text for the calling thread.  A plan
 *     is not thread-safe; distinct plans are.
 */
#ifndef COATBEM_H
#define COATBEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cb_plan_s* cb_plan;

enum {
  CB_OK = 0,
  CB_E_INVALID = -1,     /* bad argument (range, null pointer, size) */
  CB_E_NOMEM = -2,       /* device or host allocation failed */
  CB_E_DEVICE = -3,      /* a HIP call failed */
  CB_E_NOCONV = -4,      /* iteration limit reached before the tolerance */
  CB_E_NONFINITE = -5,   /* NaN/Inf met in the input or during iteration */
  CB_E_STATE = -6,       /* plan in an unusable state */
  CB_E_UNSUPPORTED = -7  /* combination not provided */
};

enum { CB_FP64 = 0, CB_FP32 = 1 };
enum { CB_DC_BZ = 0, CB_DC_ZERO = 1 };
/* How the surface operator of Eq. 1 is represented (cb_plan_opts.kernel_mode). */
enum {
  CB_KERNEL_PADDED = 0,   /* the N x N patch in a 2N-zero-padded periodic cell:
                             Eq. 11 evaluated so that it equals the
                             non-periodic sum of Eq. 1 over the patch, with
                             point-sampled K^ and the DC value of dc_mode */
  CB_KERNEL_PERIODIC = 1, /* Eq. 11 literally: the surface is L-periodic, the
                             transforms have length N (no padding) and the
                             pressure has no DC component (K^(0) = 0: a
                             uniform pressure produces no displacement and u
                             has zero mean).  The mean pressure is what a
                             force-controlled solve prescribes; the approach
                             d it returns is relative to the mean surface.
                             Non-adhesive only (Eq. 12 is derived for a
                             non-periodic system) */
  CB_KERNEL_EXACT = 2     /* the non-periodic sum of Eq. 1 with each cell
                             carrying a uniform pressure: K[i][j] is the exact
                             displacement at the centre of cell i due to unit
                             pressure over cell j, the cell integral of the
                             inverse Fourier transform of K^ (Eq. 2-3, 9-11),
                             evaluated by the same 2N-padded convolution with
                             the table of those coefficients (their DFT,
                             cb_transfer_table_exact).  No DC choice and no
                             images: the patch sum is exact up to the
                             coefficients' quadrature (about 1e-12).  Needs a
                             top layer at least Delta/8 thick (thinner:
                             CB_E_UNSUPPORTED); h = 0 or a coating of the
                             substrate's material is the half-space (Love's
                             coefficients) */
};

/* Plan options; a NULL pointer selects every default. */
typedef struct {
  int precision;   /* CB_FP64 (default) or CB_FP32.  CB_FP32: cb_apply_K is
                      an FP32 convolution; the solvers keep p, u = K p, f,
                      the gap and every reduction in FP64 and run the
                      search-direction convolutions in FP32, recomputing u
                      from p with an FP64 convolution whenever the contact
                      set changes and every `chunk` iterations */
  int dc_mode;     /* CB_DC_BZ (default): the k = 0 value of the transfer
                      function makes the frequency sum equal its integral
                      over the Brillouin zone [-pi/Delta, pi/Delta]^2;
                      CB_DC_ZERO: no DC component (Eq. 11 taken literally) */
  void* stream;    /* hipStream_t to enqueue on; NULL = the null stream */
  int autotune;    /* 1: time every FFT launch-shape variant (a graph of
                      ten convolutions each) at plan creation and keep the
                      fastest for this (device, N, precision); 0 (default):
                      variant 1, unless tune_cache holds an entry */
  const char* tune_cache; /* text file of tuned choices, one line per
                      (device architecture, N, precision): read first (an
                      entry skips the timing), appended after tuning;
                      NULL: no file */
  int fft_variant; /* 0 (default): automatic as above; 1..6 force a
                      launch shape (elements per thread in the row / column
                      kernels, row-tile height): 1 (16, 16, 1x),
                      2 (16, 8, 1x), 3 (8, 16, 1x), 4 (16, 16, 2x),
                      5 (16, 32, 1x), 6 (8, 8, 2x).  All give the same
                      transform up to rounding order. */
  int kernel_mode; /* CB_KERNEL_PADDED (default), CB_KERNEL_PERIODIC or
                      CB_KERNEL_EXACT (dc_mode is then ignored) */
} cb_plan_opts;

/* Solve options; a NULL pointer selects every default. */
typedef struct {
  double tol;        /* relative residual target; <= 0: 1e-10 (FP64), 1e-8 (FP32) */
  int max_iter;      /* conjugate-gradient iteration limit per solve; <= 0: 20000 */
  int chunk;         /* longest run of iterations on the device between host
                        checks of the convergence flag (the runs adapt to
                        the residual's progress, from min(8, chunk)); <= 0:
                        16; odd values are rounded up */
  int init;          /* 0: cold start; 1: the caller's p_io is the initial
                        guess (negative values read as 0; a guess with no
                        positive value is no guess: cold start).  Cold start
                        under displacement control: p = (d - f)+ / k00;
                        under force control: p = (d0 - f)+ rescaled to F, d0
                        estimated from the profile's depth distribution and
                        the layered modulus (uniform if no such d0 exists) */
  double attach_tol; /* adhesive: a cell outside the contact attaches when
                        its gap is below -attach_tol (length); < 0: 1e-12 L
                        (FP64), 1e-9 L (FP32) */
  int max_rounds;    /* adhesive detach/attach rounds per step; <= 0: 10000 */
  int precond;       /* non-adhesive solves: -1 (default) automatic, 0 plain
                        conjugate gradients, 1 gradients preconditioned by the
                        Fourier multiplier 1/C(kh) = 2/(E1* k K^(k)), which
                        removes the layer's stiffness contrast, 2 by 1/K^(k),
                        the inverse of the operator's symbol, 3 two-phase:
                        1 for coatings >= 3x stiffer than the substrate with
                        h <= L/16, else 0, until an iteration leaves the
                        contact set unchanged, then 2.  Automatic: 2 from a
                        start close to the contact (a caller's guess, the
                        estimated force-control cold start), else 3; always
                        3 on coatings stiff and thin as above.
                        Adhesive solves (CG on the contact set): 0, 1 or 2,
                        automatic 2.  The converged pressure is the same;
                        other values: CB_E_INVALID. */
  double preload_d;  /* adhesive cb_solve_force with F <= 0: rigid approach
                        of the preload before the retraction; <= min f:
                        automatic, the approach at which the non-adhesive
                        solve carries max(4 |F|, pi dgamma L / 2) */
} cb_solve_opts;

/* Per-solve (or per-step) outcome, filled on the host. */
typedef struct {
  int status;        /* CB_OK or a CB_E_* code for this solve / step */
  int iters;         /* conjugate-gradient iterations (all rounds) */
  int rounds;        /* adhesive detach/attach rounds (0 if non-adhesive) */
  double resid;      /* final relative residual on the contact set */
  double F;          /* total force Delta^2 sum p */
  double d;          /* rigid approach (the one found, for force control) */
  double area;       /* contact area Delta^2 |S| */
  double U_el;       /* elastic energy 1/2 Delta^2 sum p u */
  double U_ad;       /* adhesion energy -dgamma * area */
  double ms;         /* wall time of the call on the host, milliseconds */
} cb_result;

/* Read-only plan facts. */
typedef struct {
  int N, M;          /* grid and padded FFT size, M = 2N */
  int precision, dc_mode;
  double L, dx, h, E1, nu1, E2, nu2, dgamma;
  double E1s, E2s;   /* reduced moduli E/(1-nu^2), Eq. 4 */
  double sigma_c;    /* Eq. 12 critical stress (0 when dgamma = 0) */
  double k00;        /* self-influence: displacement of a cell per unit
                        pressure on itself */
  double dc;         /* the k = 0 transfer value used */
  int validity_warning; /* 1 when dgamma > 0 and h < 5 Delta: Eq. 12 assumes
                        Delta << h (Sec. 2 after Eq. 12) */
  size_t workspace_bytes;
  int fft_variant;   /* FFT launch-shape variant in use (1..6) */
  double tune_us;    /* its timed convolution, microseconds (0: not timed) */
  int kernel_mode;   /* CB_KERNEL_* */
  int table_n;       /* side of the transfer quadrant cb_plan_get_table
                        returns: N + 1 (padded), N/2 + 1 (periodic) */
  int nlayers;       /* layers of the coating (1 for cb_plan_create); h, E1,
                        nu1 are the top layer's, E2, nu2 the half-space's */
  double H;          /* total coating thickness */
} cb_plan_info;

/* Most layers of a cb_plan_create_layered stack. */
#define CB_MAX_LAYERS 8

/*
 * Device arrays passed to this library (pressures, profiles, masks, displacements,
 * and the fields of cb_apply_K / cb_apply_precond) must be 16-byte aligned:
 * every device allocation is; a view that starts at an odd element offset
 * is not, and is rejected with CB_E_INVALID.
 */

/*
 * cb_plan_create -- build the operator u = K p for one grid and material.
 *   Eq. 9-11 (Sec. 2): the transfer function is evaluated in FP64 from the
 *   normalised form of Eq. 9-10 at k = sqrt(kx^2 + ky^2) on the 2N-padded
 *   frequency grid, with the DC value of opts->dc_mode; sigma_c from Eq. 12.
 *   N: power of two, 16 <= N <= 4096.  L > 0, h >= 0, E1, E2 > 0,
 *   0 <= nu < 0.5, dgamma >= 0 (0: non-adhesive).  CB_KERNEL_PERIODIC
 *   with dgamma > 0: CB_E_UNSUPPORTED.
 *   On success *out owns device tables and workspace (see cb_plan_info);
 *   on failure *out is NULL and a CB_E_* code is returned.
 */
int cb_plan_create(cb_plan* out, int N, double L, double h, double E1,
                   double nu1, double E2, double nu2, double dgamma,
                   const cb_plan_opts* opts);

/*
 * cb_plan_create_layered -- as cb_plan_create for a coating of nlayers
 *   bonded layers (h_host[i], E_host[i], nu_host[i]), i = 0 the top layer,
 *   on a half-space (Es, nus).  The paper gives the one-layer solution
 *   (Sec. 2, Eq. 5-9) and points to multi-layer systems (Sec. 1, its
 *   reference [5]); here K^(k) is the same boundary-value problem (Eq. 5-8,
 *   conditions (a)-(d), bonded interfaces) written for every layer and
 *   solved per wavenumber, with the DC value of opts->dc_mode.  For one
 *   layer it equals Eq. 9.  sigma_c (Eq. 12) uses the top layer's E*; the
 *   Eq. 12 validity flag its h.  Host arrays of nlayers values, read only
 *   during the call.  1 <= nlayers <= CB_MAX_LAYERS, every h > 0, E > 0,
 *   0 <= nu < 0.5; other arguments as cb_plan_create.  Every solve, sweep
 *   and apply entry point accepts the plan; the learned warm start gives
 *   it no guess (zeros: the solve's cold start).
 */
int cb_plan_create_layered(cb_plan* out, int N, double L, int nlayers, const double* h_host,
                           const double* E_host, const double* nu_host, double Es, double nus,
                           double dgamma, const cb_plan_opts* opts);

/* The FP64 padded-grid table of a layered stack ((N+1)^2 doubles, host),
 * as cb_transfer_table; arguments as cb_plan_create_layered. */
int cb_transfer_table_layered(int N, double L, int nlayers, const double* h_host, const double* E_host,
                              const double* nu_host, double Es, double nus, int dc_mode,
                              double* table_host, double* k00_host);

/* Release a plan and everything it owns.  NULL is accepted (no-op). */
int cb_plan_destroy(cb_plan plan);

/* Copy the plan facts into *info (host). */
int cb_plan_get_info(cb_plan plan, cb_plan_info* info);

/* Copy the FP64 transfer table T[a][b] = K^(Delta_k sqrt(a^2 + b^2)),
 * a, b in [0, n), n = cb_plan_info.table_n (host memory, row-major), DC at
 * [0][0], WITHOUT the inverse-FFT factor the device copy carries.  Padded
 * plans: n = N + 1, Delta_k = 2 pi / (2 N Delta); periodic plans:
 * n = N/2 + 1, Delta_k = 2 pi / L, T[0][0] = 0; exact plans: n = N + 1,
 * the table of cb_transfer_table_exact. */
int cb_plan_get_table(cb_plan plan, double* table_host);

/*
 * cb_transfer_table -- the same FP64 table as cb_plan_get_table, computed on
 * the host without a device or a plan (Eq. 9-11 and the DC rule of
 * dc_mode).  Arguments as cb_plan_create; table_host: (N+1)^2 doubles.
 * k00_host (nullable): the self-influence sum(T)/M^2 over the full grid.
 */
int cb_transfer_table(int N, double L, double h, double E1, double nu1,
                      double E2, double nu2, int dc_mode, double* table_host,
                      double* k00_host);

/*
 * cb_transfer_table_exact -- exact influence coefficients of uniformly
 *   loaded square cells and the table of the CB_KERNEL_EXACT plans, on the
 *   host (no device, no plan).  Eq. 1 with piecewise-constant pressure; the
 *   displacement due to a load is the inverse Fourier transform of K^ times
 *   the load's transform (Eq. 2-3, 11), K^ of Eq. 9-10.
 *   D_host (nullable): (N+1)^2 doubles, D[m][q] = displacement at the cell
 *   offset (m Delta, q Delta), m, q in [0, N], due to unit pressure over one
 *   cell (symmetric in m, q).  table_host (nullable): (N+1)^2 doubles, the
 *   2-D DFT of the 2N-periodic embedding D_circ[m] = D[|m|] (|m| < N),
 *   D_circ[N] = D[N], i.e. T[a][b] = sum_{m,q} w_m w_q D[m][q]
 *   cos(pi a m/N) cos(pi b q/N), w = 1 at 0 and N, 2 between.  At least one
 *   output.  Arguments as cb_plan_create; a top layer thinner than Delta/8
 *   (h > 0): CB_E_UNSUPPORTED.  Runs on up to 16 host threads.
 */
int cb_transfer_table_exact(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                            double* table_host, double* D_host);

/* The same for a layered stack (arguments as cb_plan_create_layered). */
int cb_transfer_table_exact_layered(int N, double L, int nlayers, const double* h_host, const double* E_host,
                                    const double* nu_host, double Es, double nus, double* table_host,
                                    double* D_host);

/* Change the stream later calls are enqueued on (hipStream_t). */
int cb_plan_set_stream(cb_plan plan, void* stream);

/*
 * cb_apply_K -- u = K p, Eq. 1 evaluated as Eq. 11 on the zero-padded
 *   (2N)^2 grid: real 2-D FFT of p, multiply by the transfer table,
 *   inverse FFT, keep the N x N patch.  p, u: device N*N of the plan type;
 *   u must not alias p.  Asynchronous on the plan stream.
 */
int cb_apply_K(cb_plan plan, const void* p, void* u);

/*
 * cb_apply_K_batch -- u_i = K_i p_i for n problems (Eq. 1 as Eq. 11 on the
 *   2N-padded grid, as cb_apply_K), packed into one launch per transform
 *   stage (up to 32 problems per launch; more are launched in groups): for
 *   small grids one convolution is set by launch latency, not by its
 *   bytes.  plans[i]: distinct padded or exact plans (not periodic) sharing N, precision, launch
 *   shape and device (materials may differ: each problem multiplies by its
 *   own transfer table and uses its own plan's intermediate).  p[i], u[i]:
 *   device N*N arrays of the plan type, u[i] not aliasing p[i].  Enqueued
 *   on plans[0]'s stream (asynchronous); the caller orders the other plans'
 *   work against it.
 */
int cb_apply_K_batch(int n, const cb_plan* plans, const void* const* p, void* const* u);

/*
 * cb_apply_K_noalloc -- cb_apply_K for callers that cannot allocate device
 *   memory: code under HIP graph capture, tight serving loops, harnesses
 *   that forbid hipMalloc.  No plan: the caller passes the transfer table.
 *   The call allocates nothing (no hipMalloc/hipFree, no host allocation);
 *   the FFT intermediate lives in a static device array of the library
 *   (16.8 MB per device, held from module load until the process ends).
 *   N: power of two in [16, 1024] (larger N: CB_E_INVALID).  precision:
 *   CB_FP64 or CB_FP32, the type of table, p and u.  table: device,
 *   (N+1)^2 values T[a][b] = K^(dk sqrt(a^2+b^2)) / M^2, M = 2N, row-major
 *   (cb_transfer_table's table times 1/M^2, converted to the precision;
 *   cb_transfer_table_exact's table the same way gives the exact kernel).
 *   p, u: device N*N; u must not alias p; all three 16-byte aligned.
 *   stream: hipStream_t (NULL: the null stream); asynchronous.  Every call
 *   on one device shares that device's intermediate: calls that overlap
 *   on one device race and must be ordered by the caller.
 */
int cb_apply_K_noalloc(int N, int precision, const void* table, const void* p, void* u, void* stream);

/*
 * cb_apply_K_stages -- diagnostic form of cb_apply_K that launches only the
 *   stages selected in stage_mask: 1 = forward row transform (p -> plan
 *   intermediate), 2 = column transform with the transfer multiply (in place
 *   on the intermediate), 4 = inverse row transform (intermediate -> u).
 *   stage_mask = 7 is cb_apply_K.  For timing single kernels; p or u may be
 *   NULL when the stages that use them are not selected.
 */
int cb_apply_K_stages(cb_plan plan, const void* p, void* u, int stage_mask);

/*
 * cb_apply_precond -- y = M^-1 x, the solver's Fourier preconditioner (not
 *   part of the paper): the N-periodic convolution (real 2-D FFT of length
 *   N per axis, no zero padding) with the symbol s(k), k = (2 pi / L) |(a, b)|:
 *   which = 1: s = 1 / C(k h), C = E1* k K^(k) / 2 (the layer's stiffness
 *   contrast removed); which = 2: s = 1 / K^(k) (the operator's inverse
 *   symbol; at k = 0 the inverse of the padded table's DC value).  x, y:
 *   device N*N of the plan type; y must not alias x.  Asynchronous on the
 *   plan stream.  Other `which`: CB_E_INVALID.
 */
int cb_apply_precond(cb_plan plan, int which, const void* x, void* y);

/*
 * cb_solve_indent -- non-adhesive (dgamma = 0) or adhesive (dgamma > 0)
 *   contact at prescribed rigid approach d.
 *   Non-adhesive: the complementarity problem p >= 0, g >= 0, p g = 0 by
 *   constrained conjugate gradients (Sec. 2 after Eq. 11).  Adhesive: start
 *   from the geometric overlap {f <= d}, solve on the contact set, detach
 *   boundary cells whose tension exceeds sigma_c (Eq. 12), attach
 *   penetrating cells, repeat until nothing changes (Sec. 2, last
 *   paragraph).
 *   f: profile; p_io: output pressure (input guess when opts->init = 1);
 *   mask_io: optional (NULL) output contact set.  res: host, required.
 */
int cb_solve_indent(cb_plan plan, const double* f, double d, double* p_io,
                    unsigned char* mask_io, const cb_solve_opts* opts,
                    cb_result* res);

/*
 * cb_solve_force -- contact at prescribed total force F > 0;
 *   res->d returns the approach found.  Non-adhesive plans: the constrained
 *   conjugate gradients with the mean-gap shift (Sec. 2, after Eq. 11).
 *   Adhesive plans (stable branch): the approach d whose single adhesive
 *   solve (as cb_solve_indent: geometric overlap, then the Eq. 12 detach
 *   rounds) carries F, found by a bracketed regula falsi over such solves
 *   from the non-adhesive approach for F.  F(d) steps where a cell attaches
 *   or detaches, so the force is met to 1e-6 F or, where a step lies across
 *   F, to the nearer side of that step; on a coarse grid F(d) also drops
 *   where a ring of cells detaches, and then several approaches carry F:
 *   the search returns the one its bracket closes on.  res->F is the force reached,
 *   p_io / mask_io the solve at res->d, res->iters and res->rounds the
 *   totals over all solves of the search; no bracket within 60 doublings:
 *   CB_E_NOCONV.
 *   Adhesive plans, F <= 0 (pull-off under force control, Sec. 3.1, Eq. 19):
 *   preload by the single adhesive solve at opts->preload_d, then the
 *   paper's quasi-static retraction in displacement steps of
 *   (preload_d - min f) / 32, each step carrying the contact set and the
 *   pressure (as cb_sweep).  While the force keeps falling these are the
 *   states a force-controlled unloading passes through; in the first step
 *   whose force is at or below F the approach carrying F is found by
 *   regula falsi over single steps from the state of the step before (to
 *   1e-6 of max(|F|, 1e-3 x the preload force), or the nearer side of a
 *   detachment jump).  If the contact is
 *   lost first, F lies below the pull-off force: CB_E_NOCONV, with p_io /
 *   mask_io / res the step of the lowest force met (res->F is the
 *   force-controlled pull-off force to within one step).  Non-adhesive
 *   plans need F >= 0.
 */
int cb_solve_force(cb_plan plan, const double* f, double F, double* p_io,
                   unsigned char* mask_io, const cb_solve_opts* opts,
                   cb_result* res);

/*
 * cb_sweep -- quasi-static displacement-controlled adhesive approach and
 *   pull-off (Sec. 2, last paragraph): for each d_steps_host[k] attach
 *   penetrating cells, then {solve on the contact set; detach boundary
 *   cells with p < -sigma_c} until no change.  The state (p_state,
 *   mask_state) is carried between steps and left in the caller's arrays,
 *   so a sweep can be resumed by calling again with the same state.
 *   Zero both for a fresh start.  per_step_host: nsteps results.
 */
int cb_sweep(cb_plan plan, const double* f, const double* d_steps_host,
             int nsteps, double* p_state, unsigned char* mask_state,
             const cb_solve_opts* opts, cb_result* per_step_host);

/*
 * cb_solve_batch -- n independent contact problems solved concurrently.
 *   Problem i uses plans[i] (grid sizes and materials may differ; distinct
 *   plans are required), profile f[i] and pressure p_io[i] (device, double,
 *   plans[i]'s N x N), target[i] and mode[i]: 0 = prescribed approach d
 *   (cb_solve_indent; adhesive plans use the adhesive procedure), 1 =
 *   prescribed force F (cb_solve_force).  Every problem runs its own
 *   graph-captured iteration chunks on its plan's stream; up to `workers`
 *   problems (<= 0: 16) are in flight at once.  They start in order of
 *   expected length: larger N^2 first; within one N, adhesive approach
 *   steps, then stiff thin coatings (E1* >= 3 E2*, h <= L/16) by
 *   decreasing ratio of E1* to E2*, then the rest in the given order.
 *   opts (nullable) applies to every problem.  out_host: n results, each
 *   with its own status.  Returns CB_OK if every problem succeeded, else
 *   the first failing status in problem order.  Blocks until all are done.
 */
int cb_solve_batch(int n, const cb_plan* plans, const double* const* f,
                   const double* target, const int* mode, double* const* p_io,
                   const cb_solve_opts* opts, int workers, cb_result* out_host);

/*
 * cb_sweep_batch -- n independent quasi-static sweeps (cb_sweep, Sec. 2 last
 *   paragraph) run concurrently, each on its own plan's stream: problem i
 *   uses plans[i] (adhesive; distinct plans required), f[i],
 *   d_steps_host[i] (nsteps[i] approaches, host), its state
 *   p_state[i] / mask_state[i] (device, carried in and out as in cb_sweep)
 *   and per_step_host[i] (nsteps[i] results, host).  Up to `workers`
 *   (<= 0: 16) sweeps are in flight, the largest N^2 x nsteps first.
 *   Returns CB_OK if every sweep succeeded, else the first failing status
 *   in problem order.  Blocks until all are done.
 */
int cb_sweep_batch(int n, const cb_plan* plans, const double* const* f, const double* const* d_steps_host,
                   const int* nsteps, double* const* p_state, unsigned char* const* mask_state,
                   const cb_solve_opts* opts, int workers, cb_result* const* per_step_host);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper).  A small U-Net maps the
 * indenter profile and the problem scalars, on a G x G grid, to an initial
 * pressure field for the constrained conjugate-gradient solve (the
 * non-adhesive procedure of Sec. 3); only the solve it seeds decides the
 * result, so a poor guess costs iterations, never accuracy.
 *   Network: 16 channels, twelve 3x3 convolutions (two per level on G,
 *   G/2, G/4, G/8 with 2x2 average pooling, three decoder convolutions
 *   after nearest 2x upsampling with the encoder output added before the
 *   ReLU, one head convolution); q = softplus(z), p^ = q / mean(q).
 *   Training loss per sample: sum (p^ - t)^2 / sum t^2, t the solved
 *   pressure normalised to unit mean, averaged over the batch.
 *   Parameters: cb_net_num_params() floats, per layer 9*16*16 weights
 *   W[tap][co][ci] (tap = 3 (dy+1) + (dx+1)) then 16 biases.
 *   Activations: NHWC, 16 channels; x inputs are float (n, G, G, 16).
 * Activations are BF16 and every convolution runs on the BF16 matrix
 * cores with FP32 accumulation; master weights, gradients and Adam state
 * are FP32.  All pointers are device pointers unless named _host; a net
 * is not thread-safe and owns its buffers (sized at creation).
 * ------------------------------------------------------------------------ */
typedef struct cb_net_s* cb_net;

/* Number of parameters (floats). */
int cb_net_num_params(void);

/* Create a net for batches of up to `batch` samples on an H x W grid
 * (multiples of 32 in [32, 4096]) working on `stream` (NULL: the default
 * stream).  Parameters start at zero: call cb_net_set_params. */
int cb_net_create(cb_net* out, int batch, int H, int W, void* stream);
int cb_net_destroy(cb_net net);

/* Copy the FP32 parameters in (resets the Adam state and step) / out. */
int cb_net_set_params(cb_net net, const float* params);
int cb_net_get_params(cb_net net, float* params);

/* Forward pass of n <= batch samples x (n, H, W, 16); z16 (n, H, W, 16)
 * receives the head output (channel 0 is z), may be NULL.  Asynchronous. */
int cb_net_forward(cb_net net, int n, const float* x, float* z16);

/* Loss and parameter gradient for inputs x (n, H, W, 16) and targets
 * t (n, H, W); grad (cb_net_num_params floats) may be NULL, the gradient
 * is also kept for cb_net_adam_step.  Synchronises the stream. */
int cb_net_loss_grad(cb_net net, int n, const float* x, const float* t,
                     double* loss_host, float* grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the kept gradient. */
int cb_net_adam_step(cb_net net, float lr);

/* Input features of one problem on the net grid (H = W = G): the profile
 * f (Nf x Nf, Nf a multiple or a divisor of G) as its gap to the lowest
 * point, cell-averaged or repeated onto G x G and clipped at three
 * scales (0.005, 0.02, 0.08) L, plus the scalars log10(h/L)/3,
 * log10(E1/E2)/2, 2 nu1, 2 nu2, log10(F/(E2* L^2))/4 and 1 broadcast.
 * x: (G, G, 16) float.  Asynchronous. */
int cb_net_features(cb_net net, const double* f, int Nf, double L, double h,
                    double E1, double nu1, double E2, double nu2, double F,
                    float* x);

/* Warm start for a force-controlled solve on `plan`: features, forward
 * pass, q normalised to unit mean with values below `cut` set to zero,
 * interpolated (bilinear, cell-centred) or averaged onto the plan's
 * N x N grid into p_out (double).  Pass p_out to cb_solve_force with
 * opts.init = 1.  Plans of coatings >= 3x stiffer than the substrate with
 * h <= L/16 get no guess (zeros, which the solve takes as a cold start):
 * there the network's guess measured slower than a cold start.
 * Synchronises the net's stream. */
int cb_net_warmstart(cb_net net, cb_plan plan, const double* f, double F,
                     double cut, double* p_out);

/* The same for n <= batch problems at once (one forward pass of n
 * samples): plans[i], f[i] (plans[i]'s N x N), F_host[i], p_out[i].
 * Synchronises the net's stream. */
int cb_net_warmstart_batch(cb_net net, int n, const cb_plan* plans,
                           const double* const* f, const double* F_host,
                           double cut, double* const* p_out);

/* Status text; cb_last_error: last error message of this thread. */
const char* cb_status_string(int status);
const char* cb_last_error(void);
int cb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* COATBEM_H */
