// Plan construction: parameter checks, the FP64 transfer table of Eq. 9-11
// with its DC value, twiddle tables, device workspace.
#include <algorithm>
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

}  // namespace

// n-point Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on
// P_n (three-term recurrence).
void cb::gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
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

namespace {

using cb::gauss_legendre;

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
  // Phi(T) over panels graded towards t = 0 (widths doubling from 1e-6 up to
  // 0.25, then 0.25): on coatings much stiffer than the substrate C(t) has a
  // narrow peak of height about E1*/E2* at t = 0, which uniform panels
  // resolve only to about 1e-7 of the DC value
  auto phi = [&](double T) {
    const double top = T < TCUT ? T : TCUT;
    double s = 0.0, a = 0.0, b = 1e-6;
    while (a < top) {
      const double hi = b < top ? b : top;
      s += integrate([&](double t) { return shape_m1(t, c); }, a, hi, 1, x, w);
      a = hi;
      b = a < 0.25 ? 2.0 * a : a + 0.25;
    }
    return s;
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

// Integral of K^ over the Brillouin zone for a layered plan:
//   (16/E1*) [ (pi/D) ln(1+sqrt 2) + int_0^{pi/4} Phi(K(th)) dth ],
//   Phi(K) = int_0^K (C(k) - 1) dk,  K(th) = (pi/D)/cos th,
// with C - 1 integrated over geometric panels from 1e-4/H (H the total
// thickness) to 40/h_top, beyond which it is below e^-80.
static double brillouin_integral_layered(double dx, const cb::LayerStack& S, double E1s) {
  const double kmax = M_PI / dx;
  const double base = kmax * std::log(1.0 + std::sqrt(2.0));
  double H = 0.0;
  for (double hi : S.h) H += hi;
  std::vector<double> x, w;
  gauss_legendre(20, x, w);
  auto cm1 = [&](double k) { return E1s * k * cb::layered_compliance(k, S) / 2.0 - 1.0; };
  const double k0 = 1e-4 / H, kcut = 40.0 / S.h[0];
  auto phi = [&](double K) {
    const double top = K < kcut ? K : kcut;
    double s = 0.0, a = 0.0, b = k0;
    while (a < top) {
      const double hi = b < top ? b : top;
      s += integrate(cm1, a, hi, 1, x, w);
      a = hi;
      b = a * 1.3;
    }
    return s;
  };
  double outer;
  if (kmax >= kcut) {
    outer = (M_PI / 4.0) * phi(kcut);
  } else {
    outer = integrate([&](double th) { return phi(kmax / std::cos(th)); }, 0.0, M_PI / 4.0, 16, x, w);
  }
  return 16.0 / E1s * (base + outer);
}

// T[a][b] = K^(dk sqrt(a^2 + b^2)), a, b in [0, N], dk = 2 pi / (M D): the
// normalised Eq. 9-10, or the layered compliance when S is given;
// T[0][0] per dc_mode.  k00 = sum over the full M x M grid of T, divided by
// M^2 (the self-influence of a cell).
static void build_table(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                        int dc_mode, std::vector<double>& table, double& dc, double& k00,
                        const cb::LayerStack* S = nullptr) {
  const int NC = N + 1, M = 2 * N;
  const double dx = L / N, E1s = E1 / (1.0 - nu1 * nu1);
  const Coef c = coefficients(E1, nu1, E2, nu2);
  const double dk = 2.0 * M_PI / (M * dx);
  if (S) {
    cb::layered_compliance_grid(*S, dk, NC, table);
  } else {
    table.assign((size_t)NC * NC, 0.0);
    for (int a = 0; a < NC; a++)
      for (int b = 0; b < NC; b++) {
        if (a == 0 && b == 0) continue;
        const double k = dk * std::sqrt((double)a * a + (double)b * b);
        table[(size_t)a * NC + b] = 2.0 / (E1s * k) * shape(k * h, c);
      }
  }
  // Kahan sum of K^ over the full M x M grid except k = 0, by quadrant weights
  double sum = 0.0, comp = 0.0;
  for (int a = 0; a < NC; a++) {
    for (int b = 0; b < NC; b++) {
      if (a == 0 && b == 0) continue;
      const double v = table[(size_t)a * NC + b];
      const double wgt = (a == 0 || a == N ? 1.0 : 2.0) * (b == 0 || b == N ? 1.0 : 2.0);
      const double y = wgt * v - comp;
      const double t = sum + y;
      comp = (t - sum) - y;
      sum = t;
    }
  }
  const double bz = dc_mode != CB_DC_BZ ? 0.0
                    : S ? brillouin_integral_layered(dx, *S, E1s)
                        : brillouin_integral(dx, h, E1s, c);
  dc = dc_mode == CB_DC_BZ ? bz / (dk * dk) - sum : 0.0;
  table[0] = dc;
  k00 = (sum + dc) / ((double)M * M);
}

// Eq. 11 taken literally: T[a][b] = K^((2 pi / L) sqrt(a^2 + b^2)) on the
// N-periodic grid's quadrant a, b in [0, N/2], no DC component (T[0][0] = 0);
// k00 = sum over the full N x N grid of T, divided by N^2.
static void build_periodic_table(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                                 std::vector<double>& table, double& k00, const cb::LayerStack* S = nullptr) {
  const int NP = N / 2 + 1;
  const double E1s = E1 / (1.0 - nu1 * nu1);
  const Coef c = coefficients(E1, nu1, E2, nu2);
  const double dk = 2.0 * M_PI / L;
  if (S) {
    cb::layered_compliance_grid(*S, dk, NP, table);
  } else {
    table.assign((size_t)NP * NP, 0.0);
    for (int a = 0; a < NP; a++)
      for (int b = 0; b < NP; b++) {
        if (a == 0 && b == 0) continue;
        const double k = dk * std::sqrt((double)a * a + (double)b * b);
        table[(size_t)a * NP + b] = 2.0 / (E1s * k) * shape(k * h, c);
      }
  }
  double sum = 0.0, comp = 0.0;
  for (int a = 0; a < NP; a++) {
    for (int b = 0; b < NP; b++) {
      if (a == 0 && b == 0) continue;
      const double v = table[(size_t)a * NP + b];
      const double wgt = (a == 0 || a == N / 2 ? 1.0 : 2.0) * (b == 0 || b == N / 2 ? 1.0 : 2.0);
      const double y = wgt * v - comp;
      const double t = sum + y;
      comp = (t - sum) - y;
      sum = t;
    }
  }
  table[0] = 0.0;
  k00 = sum / ((double)N * N);
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

// The stack of a one-layer plan (h = 0: the half-space alone).
static cb::LayerStack one_layer(double h, double E1, double nu1, double E2, double nu2) {
  cb::LayerStack S;
  if (h > 0.0) {
    S.h.push_back(h);
    S.E.push_back(E1);
    S.nu.push_back(nu1);
  }
  S.Es = E2;
  S.nus = nu2;
  return S;
}

static int exact_out(int rc, const std::vector<double>& T, const std::vector<double>& D, double* table_out,
                     double* D_out) {
  if (rc != CB_OK) return rc;
  if (table_out) std::memcpy(table_out, T.data(), T.size() * sizeof(double));
  if (D_out) std::memcpy(D_out, D.data(), D.size() * sizeof(double));
  return CB_OK;
}

extern "C" int cb_transfer_table_exact(int N, double L, double h, double E1, double nu1, double E2, double nu2,
                                       double* table_out, double* D_out) {
  if (!table_out && !D_out) return cb_fail(CB_E_INVALID, "null outputs");
  if (int rc = check_params(N, L, h, E1, nu1, E2, nu2, 0.0)) return rc;
  std::vector<double> D, T;
  const int rc = cb::exact_influence(N, L, one_layer(h, E1, nu1, E2, nu2), D, T);
  return exact_out(rc, T, D, table_out, D_out);
}

double cb::plan_shape(const cb_plan_s* P, double k) {
  if (!P->layered) return shape(k * P->h, coefficients(P->E1, P->nu1, P->E2, P->nu2));
  if (!(k > 0.0)) return P->E1s / P->E2s;
  return P->E1s * k * layered_compliance(k, P->stack) / 2.0;
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
                  P->d_pold, P->d_mask, P->d_mask2, P->d_det, P->d_part, P->d_state,
                  P->d_save_p[0], P->d_save_p[1], P->d_save_S[0], P->d_save_S[1]};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (P->h_state) (void)hipHostFree(P->h_state);
}

// Layered stacks: 1..CB_MAX_LAYERS layers with h > 0, E > 0, 0 <= nu < 0.5.
static int check_stack(int nlayers, const double* h, const double* E, const double* nu, double Es, double nus,
                       cb::LayerStack& S) {
  if (nlayers < 1 || nlayers > CB_MAX_LAYERS)
    return cb_fail(CB_E_INVALID, "nlayers must lie in [1, " + std::to_string(CB_MAX_LAYERS) + "]");
  if (!h || !E || !nu) return cb_fail(CB_E_INVALID, "null layer array");
  S = cb::LayerStack{};
  for (int i = 0; i < nlayers; i++) {
    if (!finite_pos(h[i]) || !finite_pos(E[i]) || !(nu[i] >= 0.0 && nu[i] < 0.5))
      return cb_fail(CB_E_INVALID, "layer " + std::to_string(i) + ": need h > 0, E > 0, 0 <= nu < 0.5");
    S.h.push_back(h[i]);
    S.E.push_back(E[i]);
    S.nu.push_back(nu[i]);
  }
  S.Es = Es;
  S.nus = nus;
  return CB_OK;
}

static int plan_create_impl(cb_plan* out, int N, double L, double h, double E1, double nu1, double E2, double nu2,
                            double dgamma, const cb_plan_opts* o, const cb::LayerStack* S);

extern "C" int cb_plan_create(cb_plan* out, int N, double L, double h, double E1, double nu1,
                              double E2, double nu2, double dgamma, const cb_plan_opts* o) {
  return plan_create_impl(out, N, L, h, E1, nu1, E2, nu2, dgamma, o, nullptr);
}

extern "C" int cb_plan_create_layered(cb_plan* out, int N, double L, int nlayers, const double* h,
                                      const double* E, const double* nu, double Es, double nus, double dgamma,
                                      const cb_plan_opts* o) {
  if (!out) return cb_fail(CB_E_INVALID, "out is NULL");
  *out = nullptr;
  cb::LayerStack S;
  if (int rc = check_stack(nlayers, h, E, nu, Es, nus, S)) return rc;
  double H = 0.0;
  for (double x : S.h) H += x;
  if (int rc = check_params(N, L, H, E[0], nu[0], Es, nus, dgamma)) return rc;
  return plan_create_impl(out, N, L, h[0], E[0], nu[0], Es, nus, dgamma, o, &S);
}

extern "C" int cb_transfer_table_exact_layered(int N, double L, int nlayers, const double* h, const double* E,
                                               const double* nu, double Es, double nus, double* table_out,
                                               double* D_out) {
  if (!table_out && !D_out) return cb_fail(CB_E_INVALID, "null outputs");
  cb::LayerStack S;
  if (int rc = check_stack(nlayers, h, E, nu, Es, nus, S)) return rc;
  if (int rc = check_params(N, L, h[0], E[0], nu[0], Es, nus, 0.0)) return rc;
  std::vector<double> D, T;
  const int rc = cb::exact_influence(N, L, S, D, T);
  return exact_out(rc, T, D, table_out, D_out);
}

extern "C" int cb_transfer_table_layered(int N, double L, int nlayers, const double* h, const double* E,
                                         const double* nu, double Es, double nus, int dc_mode, double* out,
                                         double* k00_out) {
  if (!out) return cb_fail(CB_E_INVALID, "null output");
  cb::LayerStack S;
  if (int rc = check_stack(nlayers, h, E, nu, Es, nus, S)) return rc;
  if (int rc = check_params(N, L, h[0], E[0], nu[0], Es, nus, 0.0)) return rc;
  if (dc_mode != CB_DC_BZ && dc_mode != CB_DC_ZERO) return cb_fail(CB_E_INVALID, "bad dc_mode");
  std::vector<double> t;
  double dc, k00;
  build_table(N, L, h[0], E[0], nu[0], Es, nus, dc_mode, t, dc, k00, &S);
  std::memcpy(out, t.data(), t.size() * sizeof(double));
  if (k00_out) *k00_out = k00;
  return CB_OK;
}

static int plan_create_impl(cb_plan* out, int N, double L, double h, double E1, double nu1, double E2, double nu2,
                            double dgamma, const cb_plan_opts* o, const cb::LayerStack* S) {
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
  if (opts.kernel_mode != CB_KERNEL_PADDED && opts.kernel_mode != CB_KERNEL_PERIODIC &&
      opts.kernel_mode != CB_KERNEL_EXACT)
    return cb_fail(CB_E_INVALID, "kernel_mode must be CB_KERNEL_PADDED, CB_KERNEL_PERIODIC or CB_KERNEL_EXACT");
  if (opts.kernel_mode == CB_KERNEL_PERIODIC && dgamma > 0.0)
    return cb_fail(CB_E_UNSUPPORTED, "adhesion needs a non-periodic kernel (Eq. 12 is derived for a non-periodic "
                                     "system)");

  auto* P = new (std::nothrow) cb_plan_s();
  if (!P) return cb_fail(CB_E_NOMEM, "host allocation failed");
  P->N = N;
  P->kernel_mode = opts.kernel_mode;
  const bool periodic = opts.kernel_mode == CB_KERNEL_PERIODIC;
  P->M = periodic ? N : 2 * N;
  P->table_n = periodic ? N / 2 + 1 : N + 1;
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
  P->layered = S ? 1 : 0;
  P->H = h;
  if (S) {
    P->stack = *S;
    P->H = 0.0;
    for (double x : S->h) P->H += x;
  }

  // ---- FP64 transfer table on the quadrant a, b in [0, table_n) ----------
  const int M = P->M, NC = N + 1;
  // exact plans: the table of the cell coefficients; the preconditioner's
  // inverse symbol still samples K^ (ksym: positive at every wavenumber,
  // which the transform of a truncated embedding need not be)
  std::vector<double> ksym;
  if (periodic) {
    build_periodic_table(N, L, h, E1, nu1, E2, nu2, P->table64, P->k00, S);
    P->dc = 0.0;
  } else if (opts.kernel_mode == CB_KERNEL_EXACT) {
    std::vector<double> D;
    const int rc = cb::exact_influence(N, L, S ? *S : one_layer(h, E1, nu1, E2, nu2), D, P->table64);
    if (rc != CB_OK) {
      delete P;
      return rc;
    }
    P->dc = P->table64[0];
    P->k00 = D[0];
    double dc_s, k00_s;
    build_table(N, L, h, E1, nu1, E2, nu2, CB_DC_BZ, ksym, dc_s, k00_s, S);
  } else {
    build_table(N, L, h, E1, nu1, E2, nu2, opts.dc_mode, P->table64, P->dc, P->k00, S);
  }
  const std::vector<double>& qsym = ksym.empty() ? P->table64 : ksym;

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
    const double dk = 2.0 * M_PI / L;
    std::vector<double> cgrid;
    if (S) {
      // C(k) = E1* k K^ / 2 of the stack on the periodic grid (C(0) = E1*/Es*)
      if (periodic) {
        cgrid = P->table64;
      } else {
        cb::layered_compliance_grid(*S, dk, NP, cgrid);
      }
      for (int a = 0; a < NP; a++)
        for (int b = 0; b < NP; b++) {
          const double k = dk * std::sqrt((double)a * a + (double)b * b);
          double& v = cgrid[(size_t)a * NP + b];
          v = (a == 0 && b == 0) ? P->E1s / P->E2s : P->E1s * k * v / 2.0;
        }
    }
    const Coef cf = coefficients(E1, nu1, E2, nu2);
    for (int a = 0; a < NP; a++)
      for (int b = 0; b < NP; b++) {
        const double k = dk * std::sqrt((double)a * a + (double)b * b);
        pdev[(size_t)a * NP + b] = invN / (S ? cgrid[(size_t)a * NP + b] : shape(k * h, cf));
        // a periodic plan has no DC value: its inverse symbol takes that
        // of the first harmonic there (any positive value keeps M SPD)
        qdev[(size_t)a * NP + b] =
            periodic ? invN / P->table64[(a == 0 && b == 0) ? 1 : (size_t)a * NP + b]
                     : invN / qsym[(size_t)(2 * a) * NC + 2 * b];
      }
  }
  // automatic choice from a cold start: the layer multiplier for a coating
  // at least 3x stiffer than the substrate and thin relative to the domain,
  // else none (from a caller's guess the solver takes the inverse symbol)
  P->precond_auto = (P->E1s >= 3.0 * P->E2s && P->H <= L / 16.0) ? 1 : 0;

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
  const size_t ntab = (size_t)P->table_n * P->table_n;
  alloc(&P->d_table, ntab * es);
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
  if (P->precision == CB_FP32) alloc(&P->d_table64, ntab * 8);
  alloc((void**)&P->d_mask, n2);
  alloc((void**)&P->d_mask2, n2);
  alloc((void**)&P->d_det, n2);
  if (dgamma > 0.0)
    for (int q = 0; q < 2; q++) {
      alloc((void**)&P->d_save_p[q], n2 * 8);
      alloc((void**)&P->d_save_S[q], n2);
    }
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
  I.kernel_mode = P->kernel_mode;
  I.table_n = P->table_n;
  I.nlayers = P->layered ? (int)P->stack.h.size() : 1;
  I.H = P->H;
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

extern "C" int cb_apply_K_batch(int n, const cb_plan* plans, const void* const* p, void* const* u) {
  if (n < 0 || (n > 0 && (!plans || !p || !u))) return cb_fail(CB_E_INVALID, "null argument or negative count");
  if (n == 0) return CB_OK;
  const cb_plan_s* P0 = plans[0];
  if (!P0) return cb_fail(CB_E_INVALID, "null plan");
  const int prec = P0->precision == CB_FP64 ? 0 : 1;
  for (int i = 0; i < n; i++) {
    const cb_plan_s* P = plans[i];
    if (!P || !p[i] || !u[i]) return cb_fail(CB_E_INVALID, "null plan or array in the batch");
    if (P->N != P0->N || P->precision != P0->precision || P->kernel_mode == CB_KERNEL_PERIODIC ||
        P->variant[prec] != P0->variant[prec] || P->device != P0->device)
      return cb_fail(CB_E_INVALID, "batched plans must share N, precision, launch shape and device, padded kernel");
    if (p[i] == u[i]) return cb_fail(CB_E_INVALID, "u must not alias p");
    if (!cb::aligned16(p[i]) || !cb::aligned16(u[i])) return cb_fail(CB_E_INVALID, "arrays must be 16-byte aligned");
    for (int k = 0; k < i; k++)
      if (plans[k] == P) return cb_fail(CB_E_INVALID, "a plan appears twice in the batch");
  }
  for (int i0 = 0; i0 < n; i0 += cb::CB_BATCH_MAX) {
    cb::ApplyBatch ba;
    ba.n = std::min(cb::CB_BATCH_MAX, n - i0);
    for (int q = 0; q < ba.n; q++) {
      const cb_plan_s* P = plans[i0 + q];
      ba.p[q] = p[i0 + q];
      ba.S[q] = P->d_S;
      ba.T[q] = P->d_table;
      ba.u[q] = u[i0 + q];
    }
    CB_HIP(cb::launch_apply_batch(P0, ba, P0->stream));
  }
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
