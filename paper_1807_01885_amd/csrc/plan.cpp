// Plan construction: parameter checks, the FP64 transfer table of Eq. 9-11
// with its DC value, twiddle tables, device workspace.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

// last error message of the calling thread, in a fixed buffer (setting it
// allocates nothing, so the allocation-free entry point can report errors)
static thread_local char g_last_error[512];

int cb_fail_c(int status, const char* msg) {
  std::size_t i = 0;
  for (; msg && msg[i] && i + 1 < sizeof(g_last_error); i++) g_last_error[i] = msg[i];
  g_last_error[i] = '\0';
  return status;
}

int cb_fail(int status, const std::string& msg) { return cb_fail_c(status, msg.c_str()); }

extern "C" const char* cb_last_error(void) { return g_last_error; }

extern "C" const char* cb_status_string(int s) {
  switch (s) {
    case CB_OK: return "ok";
    case CB_E_INVALID: return "invalid argument";
    case CB_E_NOMEM: return "out of memory";
    case CB_E_DEVICE: return "device error";
    case CB_E_NOCONV: return "not converged";
    case CB_E_NONFINITE: return "non-finite value";
    case CB_E_STATE: return "bad plan state";
    case CB_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

extern "C" int cb_version(void) { return 100; }

namespace {

using cb::Coef;
using cb::coefficients;
using cb::shape;

// C(t) - 1 without cancellation for large t.
inline double shape_m1(double t, const Coef& c) {
  const double e2 = std::exp(-2.0 * t), e4 = e2 * e2;
  const double den = 1.0 - (c.a + c.b + 4.0 * c.b * t * t) * e2 + c.a * c.b * e4;
  const double num = (c.a + c.b + 4.0 * c.b * t + 4.0 * c.b * t * t) * e2 - 2.0 * c.a * c.b * e4;
  return num / den;
}

// n-point Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on
// P_n (three-term recurrence).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; i++) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; k++) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; k++) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Composite Gauss-Legendre integral of f over [a, b] with `panels` panels.
template <class F>
double integrate(F f, double a, double b, int panels, const std::vector<double>& x,
                 const std::vector<double>& w) {
  double s = 0.0;
  const double hw = (b - a) / panels;
  for (int p = 0; p < panels; p++) {
    const double lo = a + p * hw, mid = lo + 0.5 * hw, half = 0.5 * hw;
    double ps = 0.0;
    for (size_t i = 0; i < x.size(); i++) ps += w[i] * f(mid + half * x[i]);
    s += ps * half;
  }
  return s;
}

// Integral of K^ over the Brillouin zone [-pi/D, pi/D]^2:
//   (16/E1*) int_0^{pi/4} int_0^{K(th)} C(k h) dk dth,  K(th) = (pi/D)/cos th
// = (16/E1*) [ (pi/D) ln(1+sqrt 2) + (1/h) int_0^{pi/4} Phi((pi h/D) sec th) dth ]
// with Phi(T) = int_0^T (C(t) - 1) dt (C - 1 decays like t^2 e^{-2t}).
double brillouin_integral(double dx, double h, double E1s, const Coef& c) {
  const double kmax = M_PI / dx;
  const double base = kmax * std::log(1.0 + std::sqrt(2.0));
  std::vector<double> x, w;
  gauss_legendre(20, x, w);
  if (h <= 0.0) {
    const double c0 = shape(0.0, c);
    return 16.0 / E1s * c0 * base;
  }
  const double TCUT = 40.0;
  auto phi = [&](double T) {
    const double top = T < TCUT ? T : TCUT;
    const int panels = (int)std::ceil(top / 0.25) + 1;
    return integrate([&](double t) { return shape_m1(t, c); }, 0.0, top, panels, x, w);
  };
  const double cth = M_PI * h / dx;
  double outer;
  if (cth >= TCUT) {
    outer = (M_PI / 4.0) * phi(TCUT);
  } else {
    outer = integrate([&](double th) { return phi(cth / std::cos(th)); }, 0.0, M_PI / 4.0, 16, x, w);
  }
  return 16.0 / E1s * (base + outer / h);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

// T[a][b] = K^(dk sqrt(a^2 + b^2)), a, b in [0, N], dk = 2 pi / (M D), the
// normalised Eq. 9-10; T[0][0] per dc_mode.  k00 = sum over the full M x M
// grid of T, divided by M^2 (the self-influence of a cell).
static void build_table(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                        int dc_mode, std::vector<double>& table, double& dc, double& k00) {
  const int NC = N + 1, M = 2 * N;
  const double dx = L / N, E1s = E1 / (1.0 - nu1 * nu1);
  const Coef c = coefficients(E1, nu1, E2, nu2);
  const double dk = 2.0 * M_PI / (M * dx);
  table.assign((size_t)NC * NC, 0.0);
  // Kahan sum of K^ over the full M x M grid except k = 0, by quadrant weights
  double sum = 0.0, comp = 0.0;
  for (int a = 0; a < NC; a++) {
    for (int b = 0; b < NC; b++) {
      if (a == 0 && b == 0) continue;
      const double k = dk * std::sqrt((double)a * a + (double)b * b);
      const double v = 2.0 / (E1s * k) * shape(k * h, c);
      table[(size_t)a * NC + b] = v;
      const double wgt = (a == 0 || a == N ? 1.0 : 2.0) * (b == 0 || b == N ? 1.0 : 2.0);
      const double y = wgt * v - comp;
      const double t = sum + y;
      comp = (t - sum) - y;
      sum = t;
    }
  }
  dc = dc_mode == CB_DC_BZ ? brillouin_integral(dx, h, E1s, c) / (dk * dk) - sum : 0.0;
  table[0] = dc;
  k00 = (sum + dc) / ((double)M * M);
}

static int check_params(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                        double dgamma) {
  if (N < 16 || N > 4096 || (N & (N - 1)))
    return cb_fail(CB_E_INVALID, "N must be a power of two in [16, 4096]");
  if (!finite_pos(L)) return cb_fail(CB_E_INVALID, "L must be finite and > 0");
  if (!std::isfinite(h) || h < 0.0) return cb_fail(CB_E_INVALID, "h must be finite and >= 0");
  if (!finite_pos(E1) || !finite_pos(E2)) return cb_fail(CB_E_INVALID, "E1, E2 must be finite and > 0");
  if (!(nu1 >= 0.0 && nu1 < 0.5) || !(nu2 >= 0.0 && nu2 < 0.5))
    return cb_fail(CB_E_INVALID, "Poisson ratios must lie in [0, 0.5)");
  if (!std::isfinite(dgamma) || dgamma < 0.0) return cb_fail(CB_E_INVALID, "dgamma must be >= 0");
  return CB_OK;
}

extern "C" int cb_transfer_table(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                                 int dc_mode, double* out, double* k00_out) {
  if (!out) return cb_fail(CB_E_INVALID, "null output");
  if (int rc = check_params(N, L, h, E1, nu1, E2, nu2, 0.0)) return rc;
  if (dc_mode != CB_DC_BZ && dc_mode != CB_DC_ZERO) return cb_fail(CB_E_INVALID, "bad dc_mode");
  std::vector<double> t;
  double dc, k00;
  build_table(N, L, h, E1, nu1, E2, nu2, dc_mode, t, dc, k00);
  std::memcpy(out, t.data(), t.size() * sizeof(double));
  if (k00_out) *k00_out = k00;
  return CB_OK;
}

std::mutex& cb::graph_mutex() {
  static std::mutex mu;
  return mu;
}

static void free_plan_memory(cb_plan_s* P) {
  {
    std::lock_guard<std::mutex> lk(cb::graph_mutex());
    for (auto& g : P->graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (hipGraphExec_t ex : P->retired) (void)hipGraphExecDestroy(ex);
    P->retired.clear();
  }
  if (P->ev_in) (void)hipEventDestroy(P->ev_in);
  for (auto& e : P->ev_state)
    if (e) (void)hipEventDestroy(e);
  if (P->istream) (void)hipStreamDestroy(P->istream);
  void* ptrs[] = {P->d_table, P->d_table64, P->d_ptable, P->d_pinv, P->d_y, P->d_S, P->d_u, P->d_t, P->d_r, P->d_g,
                  P->d_pold, P->d_mask, P->d_mask2, P->d_det, P->d_part, P->d_state};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (P->h_state) (void)hipHostFree(P->h_state);
}

extern "C" int cb_plan_create(cb_plan* out, int N, double L, double h, double E1, double nu1,
                              double E2, double nu2, double dgamma, const cb_plan_opts* o) {
  if (!out) return cb_fail(CB_E_INVALID, "out is NULL");
  *out = nullptr;
  if (int rc = check_params(N, L, h, E1, nu1, E2, nu2, dgamma)) return rc;
  cb_plan_opts opts{};
  if (o) opts = *o;
  if (opts.precision != CB_FP64 && opts.precision != CB_FP32)
    return cb_fail(CB_E_INVALID, "precision must be CB_FP64 or CB_FP32");
  if (opts.dc_mode != CB_DC_BZ && opts.dc_mode != CB_DC_ZERO)
    return cb_fail(CB_E_INVALID, "dc_mode must be CB_DC_BZ or CB_DC_ZERO");
  if (opts.autotune != 0 && opts.autotune != 1) return cb_fail(CB_E_INVALID, "autotune must be 0 or 1");
  if (opts.fft_variant < 0 || opts.fft_variant > cb::CB_FFT_VARIANTS)
    return cb_fail(CB_E_INVALID, "fft_variant must be 0 (automatic) or 1.." + std::to_string(cb::CB_FFT_VARIANTS));

  auto* P = new (std::nothrow) cb_plan_s();
  if (!P) return cb_fail(CB_E_NOMEM, "host allocation failed");
  P->N = N;
  P->M = 2 * N;
  P->log2n = 0;
  while ((1 << P->log2n) < N) P->log2n++;
  P->precision = opts.precision;
  P->dc_mode = opts.dc_mode;
  P->L = L;
  P->dx = L / N;
  P->h = h;
  P->E1 = E1;
  P->nu1 = nu1;
  P->E2 = E2;
  P->nu2 = nu2;
  P->dgamma = dgamma;
  P->E1s = E1 / (1.0 - nu1 * nu1);
  P->E2s = E2 / (1.0 - nu2 * nu2);
  P->stream = (hipStream_t)opts.stream;
  // Eq. 12
  P->sigma_c = dgamma > 0.0 ? std::sqrt(P->E1s * dgamma / (0.473201 * P->dx)) : 0.0;
  P->validity_warning = (dgamma > 0.0 && h < 5.0 * P->dx) ? 1 : 0;

  // ---- FP64 transfer table on the quadrant a, b in [0, N] ----------------
  const int M = P->M, NC = N + 1;
  build_table(N, L, h, E1, nu1, E2, nu2, opts.dc_mode, P->table64, P->dc, P->k00);

  // ---- device memory ---------------------------------------------------------
  const size_t es = P->precision == CB_FP64 ? 8 : 4;
  std::vector<double> tdev(P->table64);
  const double inv = 1.0 / ((double)M * M);
  for (double& v : tdev) v *= inv;
  // Preconditioner symbols of the constrained CG, applied as N-periodic
  // convolutions (real transforms of length N, a (N/2+1)^2 quadrant with
  // 1/N^2 folded in; measured no more iterations than the padded form at a
  // third of its cost).  Wavenumbers k = (2 pi / L) |(a, b)|, which are the
  // padded grid's at (2a, 2b).
  //  - 1 / C(k h), C = E1* k K^ / 2: the ratio of the homogeneous-coating
  //    kernel to the layered one (tends to 1 at high k);
  //  - 1 / K^(k): the inverse of the operator itself, which undoes the 1/k
  //    decay of the half-space kernel as well as the layer's stiffness
  //    contrast (the padded table's DC value at k = 0).
  const int NP = N / 2 + 1;
  const double invN = 1.0 / ((double)N * N);
  std::vector<double> pdev((size_t)NP * NP), qdev((size_t)NP * NP);
  {
    const Coef cf = coefficients(E1, nu1, E2, nu2);
    const double dk = 2.0 * M_PI / L;
    for (int a = 0; a < NP; a++)
      for (int b = 0; b < NP; b++) {
        const double k = dk * std::sqrt((double)a * a + (double)b * b);
        pdev[(size_t)a * NP + b] = invN / shape(k * h, cf);
        qdev[(size_t)a * NP + b] = invN / P->table64[(size_t)(2 * a) * NC + 2 * b];
      }
  }
  // automatic choice from a cold start: the layer multiplier for a coating
  // at least 3x stiffer than the substrate and thin relative to the domain,
  // else none (from a caller's guess the solver takes the inverse symbol)
  P->precond_auto = (P->E1s >= 3.0 * P->E2s && h <= L / 16.0) ? 1 : 0;

  const size_t n2 = (size_t)N * N;
  int rc = CB_OK;
  auto alloc = [&](void** ptr, size_t bytes) {
    if (rc != CB_OK) return;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
      rc = cb_fail(CB_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      return;
    }
    P->workspace_bytes += bytes;
  };
  (void)hipGetDevice(&P->device);
  {
    const long long n = (long long)N * N;
    long long nb = (n + 1023) / 1024;
    P->nbr = (int)(nb < SOLVER_BLOCKS_MAX ? (nb < 1 ? 1 : nb) : SOLVER_BLOCKS_MAX);
  }
  alloc(&P->d_table, (size_t)NC * NC * es);
  alloc(&P->d_ptable, (size_t)NP * NP * es);
  alloc(&P->d_pinv, (size_t)NP * NP * es);
  // the intermediate and the solver arrays are sized for FP64 in both
  // precisions: solves keep their state (p, u, f, gap) in FP64 and FP32
  // plans refresh u with an FP64 convolution
  alloc(&P->d_S, cb::intermediate_elems(N) * 2 * 8);
  alloc(&P->d_u, n2 * 8);
  alloc(&P->d_t, n2 * 8);
  alloc(&P->d_r, n2 * 8);
  alloc(&P->d_g, n2 * 8);
  alloc(&P->d_pold, n2 * 8);
  alloc(&P->d_y, n2 * 8);
  if (P->precision == CB_FP32) alloc(&P->d_table64, (size_t)NC * NC * 8);
  alloc((void**)&P->d_mask, n2);
  alloc((void**)&P->d_mask2, n2);
  alloc((void**)&P->d_det, n2);
  // partial-sum regions | 32 scratch doubles
  const size_t part_doubles = (size_t)SCRATCH_OFF + 32;
  alloc((void**)&P->d_part, part_doubles * sizeof(double));
  alloc((void**)&P->d_state, sizeof(SolverState));
  if (rc == CB_OK && hipHostMalloc((void**)&P->h_state, 2 * sizeof(SolverState), 0) != hipSuccess)
    rc = cb_fail(CB_E_NOMEM, "hipHostMalloc failed");
  if (rc == CB_OK) {
    hipError_t e1, e2;
    if (P->precision == CB_FP64) {
      e1 = hipMemcpy(P->d_table, tdev.data(), tdev.size() * 8, hipMemcpyHostToDevice);
      e2 = hipMemcpy(P->d_ptable, pdev.data(), pdev.size() * 8, hipMemcpyHostToDevice);
      if (e2 == hipSuccess) e2 = hipMemcpy(P->d_pinv, qdev.data(), qdev.size() * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<float> tf(tdev.begin(), tdev.end()), pf(pdev.begin(), pdev.end());
      e1 = hipMemcpy(P->d_table, tf.data(), tf.size() * 4, hipMemcpyHostToDevice);
      if (e1 == hipSuccess)
        e1 = hipMemcpy(P->d_table64, tdev.data(), tdev.size() * 8, hipMemcpyHostToDevice);
      e2 = hipMemcpy(P->d_ptable, pf.data(), pf.size() * 4, hipMemcpyHostToDevice);
      std::vector<float> qf(qdev.begin(), qdev.end());
      if (e2 == hipSuccess) e2 = hipMemcpy(P->d_pinv, qf.data(), qf.size() * 4, hipMemcpyHostToDevice);
    }
    const hipError_t e3 = hipMemset(P->d_part, 0, part_doubles * sizeof(double));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
      rc = cb_fail(CB_E_DEVICE, "table upload failed");
  }
  if (rc == CB_OK) cb::prepare_apply(P->log2n);
  if (rc == CB_OK) {
    // default priority, no implicit sync with the null stream
    if (hipStreamCreateWithFlags(&P->istream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_state[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_state[1], hipEventDisableTiming) != hipSuccess)
      rc = cb_fail(CB_E_DEVICE, "stream/event creation failed");
  }
  if (rc == CB_OK) {
    if (opts.fft_variant > 0) {
      const int v = opts.fft_variant - 1;
      // the FP64 refresh convolutions of FP32 plans use the same shape
      // when it fits, else the default
      if (!cb::fft_variant_fits(v, P->log2n, P->precision == CB_FP64 ? 0 : 1, P->device))
        rc = cb_fail(CB_E_UNSUPPORTED, "fft_variant " + std::to_string(opts.fft_variant) +
                                           " needs more LDS per block than the device has at this N");
      P->variant[P->precision == CB_FP64 ? 0 : 1] = v;
      if (P->precision == CB_FP32 && cb::fft_variant_fits(v, P->log2n, 0, P->device)) P->variant[0] = v;
    } else {
      rc = cb::autotune_fft(P, opts.autotune, opts.tune_cache);
    }
  }
  if (rc != CB_OK) {
    free_plan_memory(P);
    delete P;
    return rc;
  }
  *out = P;
  return CB_OK;
}

extern "C" int cb_plan_destroy(cb_plan P) {
  if (!P) return CB_OK;
  if (P->istream) (void)hipStreamSynchronize(P->istream);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  free_plan_memory(P);
  delete P;
  return CB_OK;
}

extern "C" int cb_plan_get_info(cb_plan P, cb_plan_info* info) {
  if (!P || !info) return cb_fail(CB_E_INVALID, "null plan or info");
  cb_plan_info I{};
  I.N = P->N;
  I.M = P->M;
  I.precision = P->precision;
  I.dc_mode = P->dc_mode;
  I.L = P->L;
  I.dx = P->dx;
  I.h = P->h;
  I.E1 = P->E1;
  I.nu1 = P->nu1;
  I.E2 = P->E2;
  I.nu2 = P->nu2;
  I.dgamma = P->dgamma;
  I.E1s = P->E1s;
  I.E2s = P->E2s;
  I.sigma_c = P->sigma_c;
  I.k00 = P->k00;
  I.dc = P->dc;
  I.validity_warning = P->validity_warning;
  I.workspace_bytes = P->workspace_bytes;
  I.fft_variant = P->variant[P->precision == CB_FP64 ? 0 : 1] + 1;
  I.tune_us = P->tune_us;
  *info = I;
  return CB_OK;
}

extern "C" int cb_plan_get_table(cb_plan P, double* out) {
  if (!P || !out) return cb_fail(CB_E_INVALID, "null plan or output");
  std::memcpy(out, P->table64.data(), P->table64.size() * sizeof(double));
  return CB_OK;
}

extern "C" int cb_plan_set_stream(cb_plan P, void* stream) {
  if (!P) return cb_fail(CB_E_INVALID, "null plan");
  P->stream = (hipStream_t)stream;
  return CB_OK;
}

extern "C" int cb_apply_K(cb_plan P, const void* p, void* u) {
  if (!P) return cb_fail(CB_E_INVALID, "null plan");
  if (!p || !u) return cb_fail(CB_E_INVALID, "null array");
  if (p == u) return cb_fail(CB_E_INVALID, "u must not alias p");
  if (!cb::aligned16(p) || !cb::aligned16(u)) return cb_fail(CB_E_INVALID, "p and u must be 16-byte aligned");
  CB_HIP(cb::launch_apply(P, p, u, P->stream));
  return CB_OK;
}

extern "C" int cb_apply_precond(cb_plan P, int which, const void* x, void* y) {
  if (!P) return cb_fail(CB_E_INVALID, "null plan");
  if (which != 1 && which != 2) return cb_fail(CB_E_INVALID, "which must be 1 or 2");
  if (!x || !y) return cb_fail(CB_E_INVALID, "null array");
  if (!cb::aligned16(x) || !cb::aligned16(y)) return cb_fail(CB_E_INVALID, "x and y must be 16-byte aligned");
  CB_HIP(cb::launch_apply(P, x, y, P->stream, 15, nullptr, which == 1 ? P->d_ptable : P->d_pinv));
  return CB_OK;
}

extern "C" int cb_apply_K_stages(cb_plan P, const void* p, void* u, int stages) {
  if (!P) return cb_fail(CB_E_INVALID, "null plan");
  if (stages < 0 || stages > 7) return cb_fail(CB_E_INVALID, "stage_mask must be in [0, 7]");
  if (((stages & 1) && !p) || ((stages & 4) && !u)) return cb_fail(CB_E_INVALID, "null array");
  if (!cb::aligned16(p) || !cb::aligned16(u)) return cb_fail(CB_E_INVALID, "p and u must be 16-byte aligned");
  CB_HIP(cb::launch_apply(P, p, u, P->stream, stages));
  return CB_OK;
}
