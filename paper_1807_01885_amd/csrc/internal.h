// Internal plan state and launch entry points of libcoatbem.
#pragma once
#include <cmath>
#include <cstdint>
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/coatbem.h"

// Device-resident scalar state of one iterative solve.  The host writes the
// inputs before a solve; kernels carry the iteration scalars so that a whole
// chunk of iterations runs (as one captured graph) without host traffic.
struct SolverState {
  // inputs
  double tol;        // relative residual target
  double Ftarget;    // force control: total force
  double dA;         // cell area Delta^2
  double k00;        // self-influence (fallback step length 1/k00)
  double d_in;       // displacement control: rigid approach
  int force;         // 1: force control
  int pad0;
  // carried / outputs
  double d;          // rigid approach (found under force control)
  double gbar;       // force control: shift used by the next gap kernel
  double gdev;       // stored gap minus true gap in the current iteration
  double resid;      // relative residual of the last check
  double bnorm;      // fixed-set CG: ||b||
  double nact;       // |Ic| of the current iteration
  double theta;      // activation threshold (residual level) of the iteration
  double gnorm2;     // preconditioned method: sum over Ic of (g - mean)^2
  double act_scale;  // step scale for activated cells: 1, or for the
                     // preconditioned method (g . M^-1 g) / (g . g)
  double pscale;     // force control: load rescale of p and u decided at the
                     // end of an iteration, applied by the next gap kernel
  // skip_u, done, zero are adjacent: a convolution kernel given &skip_u
  // returns if either of the first two is set, given &done if done is set
  int skip_u;        // 1: u was updated linearly, its recomputation is skipped
  int done;          // 1 once converged: kernels of later iterations return
  int zero;          // always 0
  int iters;         // iterations performed
  int nonfinite;     // 1 if a NaN/Inf was met
  int breakdown;     // fixed-set CG: non-positive curvature met
  int phase;         // two-phase constrained CG: 0 before, 1 after the switch
                     // to the inverse-symbol preconditioner
  int quiet;         // consecutive iterations without a change of the contact set
  int switch_it;     // iteration count at the switch
  int pskip[4];      // FFT skip pairs of the two direction blocks:
                     // {phase-0 block idle, 0, phase-1 block idle, 0}
};

// Partial-sum regions (doubles) in the plan's reduction buffer: each holds
// an 8-double header and up to RED_BLOCKS_MAX x 8 block partials.
enum {
  R_GAP0 = 0, R_GAP1, R_STEP, R_UPD, R_RR0, R_RR1, R_ZQ, R_INIT, R_MISC, R_PZ0, R_PZ1, R_RY0, R_RY1, R_NUM
};
// partials of the solver kernels (<= 256 blocks) and of the inverse row
// transforms that carry a reduction (N / row tile blocks, up to 2048)
constexpr int RED_BLOCKS_MAX = 2048;
// blocks of the solver's elementwise kernels: at most one 512-thread block
// per CU (more lost throughput when concurrent solves share the GPU)
constexpr int SOLVER_BLOCKS_MAX = 256;
constexpr int REG_STRIDE = 8 + 8 * RED_BLOCKS_MAX;
constexpr int SCRATCH_OFF = R_NUM * REG_STRIDE;   // 32 doubles of host-read results

struct GraphEntry {
  int kind = -1;          // 0: constrained CG chunk, 1: fixed-set CG chunk
  const void* a = nullptr;
  const void* b = nullptr;
  const void* c = nullptr;
  int chunk = 0;
  hipGraphExec_t exec = nullptr;
  unsigned long long used = 0;
};
// Graph cache entries per plan.  A solve of one mode uses up to eight
// (chunk lengths 2..16, first and second phase); an adhesive force search
// adds the fixed-set solves of both contact-set buffers.
constexpr int GRAPH_CACHE = 24;

namespace cb {
// FFT launch-shape variants: complex elements per thread in the row
// kernels (K1/K3) and in the column kernel (K2), and the multiplier of the
// row-tile height (4 rows FP32, 2 rows FP64).  Variant 0 is the default.
struct FftVariant {
  int e_rows, e_cols, tile_mul;
};
constexpr int CB_FFT_VARIANTS = 6;
constexpr FftVariant kFftVariants[CB_FFT_VARIANTS] = {
    {16, 16, 1}, {16, 8, 1}, {8, 16, 1}, {16, 16, 2}, {16, 32, 1}, {8, 8, 2}};
}  // namespace cb

namespace cb {
// A stack of bonded layers (top first) on a half-space.
struct LayerStack {
  std::vector<double> h, E, nu;
  double Es = 0.0, nus = 0.0;
};
// K^(k) of the stack (k > 0), by the per-wavenumber boundary-value problem
double layered_compliance(double k, const LayerStack& S);
// out[a][b] = K^(dk sqrt(a^2 + b^2)) for a, b in [0, n) (out[0][0] = 0)
void layered_compliance_grid(const LayerStack& S, double dk, int n, std::vector<double>& out);
// n-point Gauss-Legendre nodes and weights on [-1, 1]
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// Exact influence coefficients of uniformly loaded square cells of the
// stack S (no layers: the half-space alone), D[m][q] for cell offsets
// m, q in [0, N] ((N+1)^2 row-major), and the DFT of their 2N-periodic
// embedding, T (same layout).  CB_E_UNSUPPORTED when a coating's top layer
// is thinner than Delta/8.
int exact_influence(int N, double L, const LayerStack& S, std::vector<double>& D, std::vector<double>& T);
}  // namespace cb

struct cb_plan_s {
  int N = 0, M = 0, log2n = 0, precision = 0, dc_mode = 0;
  int kernel_mode = CB_KERNEL_PADDED;  // CB_KERNEL_PERIODIC: N-periodic operator, no DC;
                                       // CB_KERNEL_EXACT: padded, table from exact cell coefficients
  int table_n = 0;                     // side of the transfer quadrant (N+1 or N/2+1)
  int layered = 0;                     // 1: transfer function of `stack` (any number of layers)
  cb::LayerStack stack;                // layers (top first) and half-space of a layered plan
  double H = 0.0;                      // total coating thickness (h for a single layer)
  double L = 0, dx = 0, h = 0, E1 = 0, nu1 = 0, E2 = 0, nu2 = 0, dgamma = 0;
  double E1s = 0, E2s = 0, sigma_c = 0, k00 = 0, dc = 0;
  int validity_warning = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<double> table64;   // table_n^2, no inverse-FFT factor
  // device memory owned by the plan
  void* d_table = nullptr;       // table_n^2, 1/M^2 (periodic: 1/N^2) folded, plan type
  void* d_table64 = nullptr;     // FP64 copy for FP32 plans (exact refreshes)
  void* d_ptable = nullptr;      // preconditioner symbol 1/C(kh) on the N-periodic grid,
                                 // (N/2+1)^2, 1/N^2 folded
  void* d_pinv = nullptr;        // preconditioner symbol 1/K^(k), same layout
  void* d_y = nullptr;           // preconditioned residual of the fixed-set CG (8 B per cell)
  int precond_auto = 0;          // automatic preconditioner of a cold start: 0 none, 1 layer
  void* d_S = nullptr;           // N x (N+1) complex intermediate
  // solver workspace (plan type unless noted)
  void* d_u = nullptr;
  void* d_t = nullptr;
  void* d_r = nullptr;
  void* d_g = nullptr;
  void* d_pold = nullptr;
  unsigned char* d_mask = nullptr;   // scratch contact set (N*N)
  unsigned char* d_mask2 = nullptr;  // second contact-set buffer (N*N)
  unsigned char* d_det = nullptr;    // detached-in-this-step flags (N*N)
  // adhesive plans: two saved states (p, contact set) of the force-controlled
  // retraction (the step before the target, the best step)
  double* d_save_p[2] = {nullptr, nullptr};
  unsigned char* d_save_S[2] = {nullptr, nullptr};
  double* d_part = nullptr;          // partial-sum regions + scratch
  SolverState* d_state = nullptr;
  SolverState* h_state = nullptr;    // pinned host mirror (2 slots)
  size_t workspace_bytes = 0;
  int nbr = 0;                       // blocks of the reduction kernels
  hipStream_t istream = nullptr;     // plan-owned stream for captured solves
  hipEvent_t ev_in = nullptr, ev_state[2] = {nullptr, nullptr};
  GraphEntry graphs[GRAPH_CACHE];
  // executable graphs evicted from the cache; destroyed with the plan (or,
  // past a bound, after the plan's stream has drained), never while a
  // launch of theirs may still be in flight or referenced
  std::vector<hipGraphExec_t> retired;
  unsigned long long graph_clock = 0;
  int use_graphs = 1;
  int variant[2] = {0, 0};  // FFT launch-shape variant of the FP64 / FP32 convolutions
  double tune_us = 0.0;     // autotuned time of one convolution (0: not tuned)
};

namespace cb {
// Device arrays are read and written in 16-byte vectors.
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Dimensionless coefficients of the normalised Eq. 9-10: with
// mu_i = E_i / (2(1+nu_i)), alpha = mu1/mu2, kappa_i = 3 - 4 nu_i,
// A/D = -a b, B/D = 4 b, 2C/D = -(a + b).
struct Coef {
  double a, b;
};
inline Coef coefficients(double E1, double nu1, double E2, double nu2) {
  const double mu1 = E1 / (2.0 * (1.0 + nu1)), mu2 = E2 / (2.0 * (1.0 + nu2));
  const double al = mu1 / mu2, k1 = 3.0 - 4.0 * nu1, k2 = 3.0 - 4.0 * nu2;
  return {(al * k2 - k1) / (1.0 + al * k2), (al - 1.0) / (al + k1)};
}
// C(t) = E1* k K^(k) / 2 at t = k h.
inline double shape(double t, const Coef& c) {
  const double e2 = std::exp(-2.0 * t), e4 = e2 * e2;
  const double num = 1.0 + 4.0 * c.b * t * e2 - c.a * c.b * e4;
  const double den = 1.0 - (c.a + c.b + 4.0 * c.b * t * t) * e2 + c.a * c.b * e4;
  return num / den;
}
}  // namespace cb

namespace cb {
// prec: -1 the plan's precision, 0 FP64, 1 FP32 (the table defaults to the
// transfer table of that precision).  Runs the plan's FFT variant for prec.
// stages: bits 0..2 select K1..K3; bit 3 (8) runs the N-periodic
// convolution instead of the padded one, with a (N/2+1)^2 table that must
// be given (the preconditioner symbols).
// Solver work carried by the row transforms of a convolution.
// K3 (inverse rows), `mode`, on the cells it writes (x = the output): 1,
// over act: sum (g - m) t, sum x t, sum x, sum t; 2, over act: sum x,
// sum (g - m) x; m = st->gdev.  One partial per K3 block, from `region` on
// (8 + block x Q).
// K1 (forward rows), `pro`, in place of reading its input: 1, the masked
// gradient act ? g - m : 0, after the convergence check from the gap
// kernel's partials (`gap`, `nb` blocks); 2, the search direction
// t = act ? (x - xbar) + beta t : 0, written back to `tdir` and
// transformed, with x, xbar and beta those of the plain method (x = g;
// convergence check here) or of the preconditioned one (x = `x`, sums of
// the preconditioner's K3 in `pz`, `nbz` blocks), whichever the phase
// uses.  Every K1 block folds the partials itself.
struct EpiArgs {
  int mode = 0;
  int pro = 0;
  const unsigned char* act = nullptr;
  const void* g = nullptr;
  const void* t = nullptr;
  SolverState* st = nullptr;
  double* region = nullptr;
  const void* x = nullptr;
  void* tdir = nullptr;
  const double* gap = nullptr;
  const double* gap_prev = nullptr;
  const double* pz = nullptr;
  const double* pz_prev = nullptr;
  const double* upd = nullptr;
  double* gbar2 = nullptr;
  int nb = 0;
  int nbz = 0;
  int par = 0;
  int plain0 = 0;  // the first (or only) phase uses the plain direction
  int two = 0;     // two-phase solve
};
// Several padded problems of one size and precision in one launch per
// stage: problem q's input, intermediate, table (1/M^2 folded) and output.
constexpr int CB_BATCH_MAX = 32;
struct ApplyBatch {
  int n = 0;   // problems in this launch (<= CB_BATCH_MAX)
  int nb = 0;  // blocks per problem of the stage being launched
  const void* p[CB_BATCH_MAX];
  void* S[CB_BATCH_MAX];
  const void* T[CB_BATCH_MAX];
  void* u[CB_BATCH_MAX];
};
// one launch per stage for ba.n problems with plan P0's size, precision and
// launch shape
hipError_t launch_apply_batch(const cb_plan_s* P0, const ApplyBatch& ba, hipStream_t st);
hipError_t launch_apply(const cb_plan_s* P, const void* p, void* u, hipStream_t st, int stages = 7,
                        const int* skip = nullptr, const void* table = nullptr, int prec = -1,
                        const EpiArgs* epi = nullptr);
// blocks of the inverse row transform (the partials a K3 reduction writes)
int rows_blocks(const cb_plan_s* P, int prec, bool periodic);
inline size_t intermediate_elems(int N) { return (size_t)N * (N + 1); }
// dynamic-LDS attributes of every variant's kernels for this size
void prepare_apply(int log2n);
// one variant's entry points (fft.hip compiled once per variant)
#define CB_DECLARE_FFT_VARIANT(k)                                                                         \
  hipError_t launch_apply_v##k(const cb_plan_s* P, const void* p, void* u, hipStream_t st, int stages,   \
                               const int* skip, const void* table, int prec, const EpiArgs* epi);       \
  int rows_blocks_v##k(int log2n, int prec, int periodic);                                               \
  hipError_t launch_apply_batch_v##k(int log2n, int prec, const ApplyBatch& ba, hipStream_t st);          \
  void prepare_apply_v##k(int log2n);                                                                    \
  size_t lds_bytes_v##k(int log2n, int prec);
CB_DECLARE_FFT_VARIANT(0)
CB_DECLARE_FFT_VARIANT(1)
CB_DECLARE_FFT_VARIANT(2)
CB_DECLARE_FFT_VARIANT(3)
CB_DECLARE_FFT_VARIANT(4)
CB_DECLARE_FFT_VARIANT(5)
#undef CB_DECLARE_FFT_VARIANT
// 1 if variant v fits the device's LDS per block for this size and precision
bool fft_variant_fits(int v, int log2n, int prec, int device);
// time every fitting variant for the plan's precision, or take it from the cache
int autotune_fft(cb_plan_s* P, int autotune, const char* cache);
}  // namespace cb

namespace cb {
// C(k) = E1* k K^(k) / 2 of the plan's material (E1* of the top layer): the
// transfer function relative to a homogeneous half-space of the coating
double plan_shape(const cb_plan_s* P, double k);
}  // namespace cb

namespace cb {
// One process-wide lock around stream capture, graph instantiation and the
// destruction of graphs and executable graphs.  Batched solves drive many
// plans from concurrent host threads; the lock keeps those graph-management
// calls from running at the same time (launches of existing executable
// graphs and all other stream work stay unserialised).
std::mutex& graph_mutex();
}  // namespace cb

// error reporting (thread-local message)
int cb_fail(int status, const std::string& msg);
// the same without constructing a string (no allocation)
int cb_fail_c(int status, const char* msg);
#define CB_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return cb_fail(CB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
