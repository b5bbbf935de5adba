// Iterative contact solves on the device (Sec. 2 after Eq. 11, Eq. 12 and
// the pull-off procedure of Sec. 2).
//
// Non-adhesive: constrained conjugate gradients (Polonsky-Keer reading of
// the paper's reference [8]); the converged pressure solves
//   p >= 0, g = K p + f - d >= 0, p g = 0.
// Adhesive: plain conjugate gradients on the contact set S ((K p)_i = d - f_i
// on S, p = 0 off S), then the Eq. 12 detachment of boundary cells with
// tension above sigma_c and attachment of penetrating cells, repeated until
// nothing changes.
//
// Every reduction accumulates in FP64 (also for FP32 fields), per block in a
// fixed order, and the last block to finish folds the block partials in a
// fixed order and updates the device-resident SolverState: results are
// bitwise reproducible and no host round trip is needed per iteration.
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace cb {

constexpr int RED_THREADS = 256;
constexpr int MAXQ = 6;  // reduced quantities per kernel

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce Q values per thread to block totals in `out` (thread 0 holds them).
// ISMAX[q] selects max instead of sum for quantity q.
template <int Q>
__device__ __forceinline__ void block_reduce(double (&v)[Q], const bool (&ismax)[Q], double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; q++) v[q] = ismax[q] ? wave_max(v[q]) : wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < Q; q++) sh[w * Q + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr int NW = RED_THREADS / 64;
#pragma unroll
    for (int q = 0; q < Q; q++) {
      double a = sh[q];
      for (int i = 1; i < NW; i++) a = ismax[q] ? fmax(a, sh[i * Q + q]) : a + sh[i * Q + q];
      v[q] = a;
    }
  }
  __syncthreads();
}

// Write this block's partials; the last block to arrive folds all partials
// (fixed order) into tot[] and returns true in every thread of that block.
template <int Q>
__device__ bool last_block_fold(double (&v)[Q], const bool (&ismax)[Q], double* part,
                                unsigned int* counter, double (&tot)[Q], double* sh) {
  __shared__ int am_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; q++) part[blockIdx.x * Q + q] = v[q];
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return false;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  double a[Q];
#pragma unroll
  for (int q = 0; q < Q; q++) a[q] = ismax[q] ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += RED_THREADS) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const double x = __hip_atomic_load(&part[b * Q + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a[q] = ismax[q] ? fmax(a[q], x) : a[q] + x;
    }
  }
  block_reduce<Q>(a, ismax, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; q++) tot[q] = a[q];
    *counter = 0u;
  }
  return true;
}

template <typename T>
__device__ __forceinline__ bool finite_val(T x) { return isfinite(x); }

// ---------------------------------------------------------------------------
// Non-adhesive constrained CG kernels
// ---------------------------------------------------------------------------
struct KParams {
  int n;            // N*N
  int force;        // 1: force control
  double tol;
  double Ftarget;
  double dA;
  double k00;
};

// Force control: mean of u + f over Ic -> state.d (the approach)
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_mean_gap(const T* __restrict__ p, const T* __restrict__ u, const T* __restrict__ f, KParams kp,
           SolverState* st, double* part, unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64 * 2];
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, false};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    if (p[i] > T(0)) {
      v[0] += (double)u[i] + (double)f[i];
      v[1] += 1.0;
    }
  }
  block_reduce<2>(v, mx, sh);
  double tot[2];
  if (last_block_fold<2>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    if (tot[1] > 0.0) st->d = tot[0] / tot[1];
    else { st->nonfinite = 1; st->done = 1; }
  }
}

// g = u + f - d; residual check; conjugate-direction coefficient
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_gap(const T* __restrict__ p, const T* __restrict__ u, const T* __restrict__ f, T* __restrict__ g,
      KParams kp, SolverState* st, double* part, unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64 * 5];
  const double d = st->d;
  // G = sum_Ic g^2, rhs2 = sum_Ic (d-f)^2, n_Ic, max_{!Ic} (-g), nonfinite
  double v[5] = {0.0, 0.0, 0.0, -INFINITY, 0.0};
  const bool mx[5] = {false, false, false, true, true};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    const double gi = (double)u[i] + (double)f[i] - d;
    const T gt = (T)gi;
    g[i] = gt;
    if (!finite_val(gt)) v[4] = 1.0;
    if (p[i] > T(0)) {
      v[0] += (double)gt * (double)gt;
      const double r = d - (double)f[i];
      v[1] += r * r;
      v[2] += 1.0;
    } else {
      v[3] = fmax(v[3], -(double)gt);
    }
  }
  block_reduce<5>(v, mx, sh);
  double tot[5];
  if (last_block_fold<5>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    st->iters += 1;
    if (tot[4] > 0.0) { st->nonfinite = 1; st->done = 1; return; }
    const double G = tot[0];
    const double rn = sqrt(tot[1]);
    const double res = rn > 0.0 ? sqrt(G) / rn : sqrt(G);
    const double scale = rn / sqrt(fmax(tot[2], 1.0));
    st->resid = res;
    st->nactive = (int)tot[2];
    st->viol = (tot[3] > kp.tol * scale) ? 1 : 0;
    if (res <= kp.tol && !st->viol) { st->done = 1; return; }
    st->rr = (st->delta > 0.0) ? G / st->G_old : 0.0;  // beta
    st->G_old = G;
  }
}

// t = Ic ? g + beta t : 0
template <typename T>
__global__ void k_dir(const T* __restrict__ p, const T* __restrict__ g, T* __restrict__ t, int n,
                      const SolverState* st) {
  if (st->done) return;
  const T beta = (T)st->rr;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    t[i] = p[i] > T(0) ? g[i] + beta * t[i] : T(0);
}

// Force control: mean of r over Ic
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_mean_r(const T* __restrict__ p, const T* __restrict__ r, KParams kp, SolverState* st, double* part,
         unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64 * 2];
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, false};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    if (p[i] > T(0)) {
      v[0] += (double)r[i];
      v[1] += 1.0;
    }
  }
  block_reduce<2>(v, mx, sh);
  double tot[2];
  if (last_block_fold<2>(v, mx, part, counter, tot, sh) && threadIdx.x == 0)
    st->rmean = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
}

// tau = sum_Ic g t / sum_Ic (r - rmean) t
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_step(const T* __restrict__ p, const T* __restrict__ g, const T* __restrict__ t,
       const T* __restrict__ r, KParams kp, SolverState* st, double* part, unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64 * 2];
  const double rm = kp.force ? st->rmean : 0.0;
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, false};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    if (p[i] > T(0)) {
      const double ti = (double)t[i];
      v[0] += (double)g[i] * ti;
      v[1] += ((double)r[i] - rm) * ti;
    }
  }
  block_reduce<2>(v, mx, sh);
  double tot[2];
  if (last_block_fold<2>(v, mx, part, counter, tot, sh) && threadIdx.x == 0)
    st->tau = tot[1] > 0.0 ? tot[0] / tot[1] : 1.0 / kp.k00;
}

// p <- max(p - tau t, 0) on Ic; p = 0 & g < 0 -> p = -tau g (restart)
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_update(T* __restrict__ p, const T* __restrict__ g, const T* __restrict__ t, KParams kp,
         SolverState* st, double* part, unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64 * 2];
  const double tau = st->tau;
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, false};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    double pi = (double)p[i];
    if (pi > 0.0) pi = pi - tau * (double)t[i];
    T pn = (T)(pi > 0.0 ? pi : 0.0);
    const T gi = g[i];
    if (pn == T(0) && gi < T(0)) {
      pn = (T)(-tau * (double)gi);
      v[1] += 1.0;
    }
    p[i] = pn;
    v[0] += (double)pn;
  }
  block_reduce<2>(v, mx, sh);
  double tot[2];
  if (last_block_fold<2>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    st->delta = tot[1] > 0.0 ? 0.0 : 1.0;
    st->F = kp.dA * tot[0];
    st->bnorm = (kp.force && tot[0] > 0.0) ? kp.Ftarget / (kp.dA * tot[0]) : 1.0;  // rescale
  }
}

template <typename T>
__global__ void k_rescale(T* __restrict__ p, int n, const SolverState* st) {
  if (st->done) return;
  const double s = st->bnorm;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = (T)((double)p[i] * s);
}

// ---------------------------------------------------------------------------
// initial guesses, statistics, masks
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_minmax(const T* __restrict__ x, int n, double* part, unsigned* counter, double* out) {
  __shared__ double sh[RED_THREADS / 64 * 3];
  double v[3] = {-INFINITY, -INFINITY, 0.0};
  const bool mx[3] = {true, true, true};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += gridDim.x * RED_THREADS) {
    const double a = (double)x[i];
    v[0] = fmax(v[0], -a);
    v[1] = fmax(v[1], a);
    if (!isfinite(a)) v[2] = 1.0;
  }
  block_reduce<3>(v, mx, sh);
  double tot[3];
  if (last_block_fold<3>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    out[0] = -tot[0];
    out[1] = tot[1];
    out[2] = tot[2];
  }
}

// p = max(d - f, 0) / k00 (cold start at prescribed approach)
template <typename T>
__global__ void k_init_disp(T* __restrict__ p, const T* __restrict__ f, int n, double d, double k00) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double v = d - (double)f[i];
    p[i] = (T)(v > 0.0 ? v / k00 : 0.0);
  }
}
template <typename T>
__global__ void k_fill(T* __restrict__ p, int n, double v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = (T)v;
}
template <typename T>
__global__ void k_clamp_pos(T* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = p[i] > T(0) ? p[i] : T(0);
}

// F = dA sum p, area = dA |S|, U_el = dA/2 sum p u; out[0..3]: sum p, count, sum p u, nonfinite
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_stats(const T* __restrict__ p, const T* __restrict__ u, const unsigned char* __restrict__ S, int n,
        double* part, unsigned* counter, double* out) {
  __shared__ double sh[RED_THREADS / 64 * 4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const bool mx[4] = {false, false, false, true};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += gridDim.x * RED_THREADS) {
    const double pi = (double)p[i];
    v[0] += pi;
    v[1] += S ? (S[i] ? 1.0 : 0.0) : (pi > 0.0 ? 1.0 : 0.0);
    v[2] += pi * (double)u[i];
    if (!isfinite(pi)) v[3] = 1.0;
  }
  block_reduce<4>(v, mx, sh);
  double tot[4];
  if (last_block_fold<4>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 4; q++) out[q] = tot[q];
  }
}

template <typename T>
__global__ void k_mask_from_p(const T* __restrict__ p, unsigned char* __restrict__ S, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    S[i] = p[i] > T(0) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Adhesive kernels
// ---------------------------------------------------------------------------
// S0 = {f - d <= 0}, p = 0
template <typename T>
__global__ void k_mask_overlap(const T* __restrict__ f, double d, unsigned char* __restrict__ S,
                               T* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    S[i] = ((double)f[i] - d <= 0.0) ? 1 : 0;
    p[i] = T(0);
  }
}

// Start of a displacement step: S |= {f - d + u < 0}, p = 0 off S, det = 0
template <typename T>
__global__ void k_attach_start(const T* __restrict__ f, const T* __restrict__ u, double d,
                               unsigned char* __restrict__ S, unsigned char* __restrict__ det,
                               T* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const bool s = S[i] || ((double)f[i] - d + (double)u[i] < 0.0);
    S[i] = s ? 1 : 0;
    det[i] = 0;
    if (!s) p[i] = T(0);
  }
}

// Fixed-set CG: r = S ? d - f - u : 0; z = r; rr, bnorm
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_mcg_init(const T* __restrict__ f, const T* __restrict__ u, const unsigned char* __restrict__ S,
           T* __restrict__ r, T* __restrict__ z, KParams kp, SolverState* st, double* part,
           unsigned* counter) {
  __shared__ double sh[RED_THREADS / 64 * 3];
  const double d = st->d;
  double v[3] = {0.0, 0.0, 0.0};
  const bool mx[3] = {false, false, true};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    T ri = T(0);
    if (S[i]) {
      const double b = d - (double)f[i];
      ri = (T)(b - (double)u[i]);
      v[1] += b * b;
    }
    r[i] = ri;
    z[i] = ri;
    v[0] += (double)ri * (double)ri;
    if (!finite_val(ri)) v[2] = 1.0;
  }
  block_reduce<3>(v, mx, sh);
  double tot[3];
  if (last_block_fold<3>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    st->rr = tot[0];
    st->bnorm = sqrt(tot[1]);
    st->resid = st->bnorm > 0.0 ? sqrt(tot[0]) / st->bnorm : 0.0;
    if (tot[2] > 0.0) { st->nonfinite = 1; st->done = 1; }
    else if (st->bnorm == 0.0 || st->resid <= kp.tol) st->done = 1;
  }
}

// alpha = rr / sum_S z q
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_mcg_alpha(const T* __restrict__ z, const T* __restrict__ q, const unsigned char* __restrict__ S,
            KParams kp, SolverState* st, double* part, unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64];
  double v[1] = {0.0};
  const bool mx[1] = {false};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS)
    if (S[i]) v[0] += (double)z[i] * (double)q[i];
  block_reduce<1>(v, mx, sh);
  double tot[1];
  if (last_block_fold<1>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    if (tot[0] > 0.0) st->tau = st->rr / tot[0];
    else { st->tau = 0.0; st->done = 1; }
  }
}

// x += alpha z, r -= alpha q on S; beta = rr_new / rr; convergence
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_mcg_update(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ z, const T* __restrict__ q,
             const unsigned char* __restrict__ S, KParams kp, SolverState* st, double* part,
             unsigned* counter) {
  if (st->done) return;
  __shared__ double sh[RED_THREADS / 64 * 2];
  const double a = st->tau;
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, true};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < kp.n; i += gridDim.x * RED_THREADS) {
    if (S[i]) {
      x[i] = (T)((double)x[i] + a * (double)z[i]);
      const T ri = (T)((double)r[i] - a * (double)q[i]);
      r[i] = ri;
      v[0] += (double)ri * (double)ri;
      if (!finite_val(ri)) v[1] = 1.0;
    }
  }
  block_reduce<2>(v, mx, sh);
  double tot[2];
  if (last_block_fold<2>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    st->iters += 1;
    if (tot[1] > 0.0) { st->nonfinite = 1; st->done = 1; return; }
    const double rr = tot[0];
    st->G_old = st->rr > 0.0 ? rr / st->rr : 0.0;  // beta
    st->rr = rr;
    st->resid = st->bnorm > 0.0 ? sqrt(rr) / st->bnorm : 0.0;
    if (st->resid <= kp.tol) st->done = 1;
  }
}

template <typename T>
__global__ void k_mcg_dir(T* __restrict__ z, const T* __restrict__ r, const unsigned char* __restrict__ S,
                          int n, const SolverState* st) {
  if (st->done) return;
  const T beta = (T)st->G_old;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    z[i] = S[i] ? r[i] + beta * z[i] : T(0);
}

// Eq. 12 detachment of boundary cells and attachment of penetrating cells.
// Reads S_in (old set), writes S_out; out[0] = changed cells.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_detach_attach(const T* __restrict__ f, const T* __restrict__ u, T* __restrict__ p,
                const unsigned char* __restrict__ Sin, unsigned char* __restrict__ Sout,
                unsigned char* __restrict__ det, int N, double d, double sigma_c, double atol,
                double* part, unsigned* counter, int* changed) {
  __shared__ double sh[RED_THREADS / 64 * 2];
  const int n = N * N;
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, false};
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += gridDim.x * RED_THREADS) {
    const int r = i / N, c = i - r * N;
    const bool s = Sin[i] != 0;
    bool ns = s;
    if (s) {
      const bool inner = r > 0 && r < N - 1 && c > 0 && c < N - 1 && Sin[i - 1] && Sin[i + 1] &&
                         Sin[i - N] && Sin[i + N];
      if (!inner && (double)p[i] < -sigma_c) {
        ns = false;
        det[i] = 1;
        p[i] = T(0);
        v[0] += 1.0;
      }
    } else if (!det[i] && ((double)f[i] - d + (double)u[i] < -atol)) {
      ns = true;
      v[1] += 1.0;
    }
    Sout[i] = ns ? 1 : 0;
  }
  block_reduce<2>(v, mx, sh);
  double tot[2];
  if (last_block_fold<2>(v, mx, part, counter, tot, sh) && threadIdx.x == 0) {
    changed[0] = (int)tot[0];
    changed[1] = (int)tot[1];
  }
}

template <typename T>
__global__ void k_zero_off(T* __restrict__ p, const unsigned char* __restrict__ S, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (!S[i]) p[i] = T(0);
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
struct Ctx {
  cb_plan_s* P;
  hipStream_t st;
  int n;
  int nblk;          // reduction grid
  int eblk;          // elementwise grid
  unsigned* counter;
  double* part;
  double* scratch;   // small device result area (after the partials)
};

static Ctx make_ctx(cb_plan_s* P) {
  Ctx c;
  c.P = P;
  c.st = P->stream;
  c.n = P->N * P->N;
  int nb = (c.n + RED_THREADS * 4 - 1) / (RED_THREADS * 4);
  if (nb > P->nblk_red - 2) nb = P->nblk_red - 2;
  if (nb < 1) nb = 1;
  c.nblk = nb;
  c.eblk = (c.n + 255) / 256 < 2048 ? (c.n + 255) / 256 : 2048;
  // d_part: [nblk_red * 8 partials | 16 scratch doubles | counter]
  c.part = P->d_part;
  c.scratch = P->d_part + (size_t)P->nblk_red * 8;
  c.counter = reinterpret_cast<unsigned*>(P->d_part + (size_t)P->nblk_red * 8 + 24);
  return c;
}

static int sync_state(cb_plan_s* P) {
  CB_HIP(hipMemcpyAsync(P->h_state, P->d_state, sizeof(SolverState), hipMemcpyDeviceToHost, P->stream));
  CB_HIP(hipStreamSynchronize(P->stream));
  return CB_OK;
}

static int read_scratch(const Ctx& c, double* out, int k) {
  CB_HIP(hipMemcpyAsync(out, c.scratch, k * sizeof(double), hipMemcpyDeviceToHost, c.st));
  CB_HIP(hipStreamSynchronize(c.st));
  return CB_OK;
}

template <typename T>
static int apply(const Ctx& c, const void* x, void* y) {
  CB_HIP(launch_apply(c.P, x, y, c.st));
  return CB_OK;
}

// One constrained-CG iteration (enqueue only).
template <typename T>
static int pk_iteration(const Ctx& c, T* p, const T* f, const KParams& kp) {
  cb_plan_s* P = c.P;
  T* u = (T*)P->d_u;
  T* g = (T*)P->d_g;
  T* t = (T*)P->d_t;
  T* r = (T*)P->d_r;
  SolverState* st = P->d_state;
  if (kp.force)
    hipLaunchKernelGGL(k_mean_gap<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, u, f, kp, st, c.part, c.counter);
  hipLaunchKernelGGL(k_gap<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, u, f, g, kp, st, c.part, c.counter);
  hipLaunchKernelGGL(k_dir<T>, dim3(c.eblk), dim3(256), 0, c.st, p, g, t, c.n, st);
  if (int rc = apply<T>(c, t, r)) return rc;
  if (kp.force)
    hipLaunchKernelGGL(k_mean_r<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, r, kp, st, c.part, c.counter);
  hipLaunchKernelGGL(k_step<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, g, t, r, kp, st, c.part, c.counter);
  hipLaunchKernelGGL(k_update<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, g, t, kp, st, c.part, c.counter);
  if (kp.force) hipLaunchKernelGGL(k_rescale<T>, dim3(c.eblk), dim3(256), 0, c.st, p, c.n, st);
  if (int rc = apply<T>(c, p, u)) return rc;
  CB_HIP(hipGetLastError());
  return CB_OK;
}

static void fill_opts(const cb_plan_s* P, const cb_solve_opts* o, double& tol, int& max_iter, int& chunk,
                      int& init, double& atol, int& max_rounds) {
  cb_solve_opts d{};
  if (o) d = *o;
  tol = d.tol > 0 ? d.tol : (P->precision == CB_FP64 ? 1e-10 : 1e-6);
  max_iter = d.max_iter > 0 ? d.max_iter : 20000;
  chunk = d.chunk > 0 ? d.chunk : 16;
  init = d.init;
  atol = d.attach_tol >= 0 ? d.attach_tol : (P->precision == CB_FP64 ? 1e-12 : 1e-6) * P->L;
  max_rounds = d.max_rounds > 0 ? d.max_rounds : 10000;
}

static void reset_state(cb_plan_s* P, double d) {
  SolverState s{};
  s.G_old = 1.0;
  s.delta = 0.0;
  s.d = d;
  s.bnorm = 1.0;
  *P->h_state = s;
}

template <typename T>
static int pk_solve(cb_plan_s* P, const T* f, double target, bool force, T* p, unsigned char* mask,
                    const cb_solve_opts* o, cb_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c = make_ctx(P);
  double tol, atol;
  int max_iter, chunk, init, max_rounds;
  fill_opts(P, o, tol, max_iter, chunk, init, atol, max_rounds);
  const double dA = P->dx * P->dx;
  *res = cb_result{};
  // profile range and finiteness
  hipLaunchKernelGGL(k_minmax<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, f, c.n, c.part, c.counter, c.scratch);
  double mm[3];
  if (int rc = read_scratch(c, mm, 3)) return rc;  // (synchronises)
  if (mm[2] > 0.0) return cb_fail(CB_E_NONFINITE, "profile f contains NaN/Inf");
  const double fmin = mm[0];
  bool trivial = force ? !(target > 0.0) : (target <= fmin);
  if (trivial) {
    hipLaunchKernelGGL(k_fill<T>, dim3(c.eblk), dim3(256), 0, c.st, p, c.n, 0.0);
    if (mask) CB_HIP(hipMemsetAsync(mask, 0, c.n, c.st));
    CB_HIP(hipStreamSynchronize(c.st));
    res->status = CB_OK;
    res->d = force ? fmin : target;
    res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return CB_OK;
  }
  // initial pressure
  if (init == 1) {
    hipLaunchKernelGGL(k_clamp_pos<T>, dim3(c.eblk), dim3(256), 0, c.st, p, c.n);
  } else if (force) {
    hipLaunchKernelGGL(k_fill<T>, dim3(c.eblk), dim3(256), 0, c.st, p, c.n, target / (dA * c.n));
  } else {
    hipLaunchKernelGGL(k_init_disp<T>, dim3(c.eblk), dim3(256), 0, c.st, p, f, c.n, target, P->k00);
  }
  reset_state(P, force ? 0.0 : target);
  if (force) {
    // rescale to the target force
    hipLaunchKernelGGL(k_stats<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, p, (const unsigned char*)nullptr,
                       c.n, c.part, c.counter, c.scratch);
    double s4[4];
    if (int rc = read_scratch(c, s4, 4)) return rc;
    if (!(s4[0] > 0.0) || s4[3] > 0.0) return cb_fail(CB_E_NONFINITE, "initial pressure has no positive finite part");
    P->h_state->bnorm = target / (dA * s4[0]);
  }
  CB_HIP(hipMemcpyAsync(P->d_state, P->h_state, sizeof(SolverState), hipMemcpyHostToDevice, c.st));
  if (force) hipLaunchKernelGGL(k_rescale<T>, dim3(c.eblk), dim3(256), 0, c.st, p, c.n, P->d_state);
  if (int rc = apply<T>(c, p, P->d_u)) return rc;
  KParams kp{c.n, force ? 1 : 0, tol, force ? target : 0.0, dA, P->k00};
  int status = CB_E_NOCONV;
  int launched = 0;
  while (launched < max_iter) {
    const int k = chunk < max_iter - launched ? chunk : max_iter - launched;
    for (int i = 0; i < k; i++)
      if (int rc = pk_iteration<T>(c, p, f, kp)) return rc;
    launched += k;
    if (int rc = sync_state(P)) return rc;
    if (P->h_state->nonfinite) { status = CB_E_NONFINITE; break; }
    if (P->h_state->done) { status = CB_OK; break; }
  }
  if (status == CB_E_NOCONV) {
    // the last launched check may have converged
    if (P->h_state->done) status = CB_OK;
  }
  SolverState s = *P->h_state;
  hipLaunchKernelGGL(k_stats<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, p, (const T*)P->d_u,
                     (const unsigned char*)nullptr, c.n, c.part, c.counter, c.scratch);
  double s4[4];
  if (int rc = read_scratch(c, s4, 4)) return rc;
  if (mask) hipLaunchKernelGGL(k_mask_from_p<T>, dim3(c.eblk), dim3(256), 0, c.st, p, mask, c.n);
  CB_HIP(hipStreamSynchronize(c.st));
  res->status = status;
  res->iters = s.iters;
  res->rounds = 0;
  res->resid = s.resid;
  res->F = dA * s4[0];
  res->d = s.d;
  res->area = dA * s4[1];
  res->U_el = 0.5 * dA * s4[2];
  res->U_ad = 0.0;
  res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (status != CB_OK)
    return cb_fail(status, status == CB_E_NOCONV ? "iteration limit reached" : "non-finite value in iteration");
  return CB_OK;
}

// CG on the fixed set S (device mask); x in/out.  The recurrence residual
// is confirmed by a true residual b - K x after convergence; if that is
// still above tol the CG restarts from x (at most twice more).
template <typename T>
static int set_solve(const Ctx& c, const T* f, double d, const unsigned char* S, T* x, double tol,
                     int max_iter, int chunk, int& iters, double& resid) {
  cb_plan_s* P = c.P;
  T* u = (T*)P->d_u;
  T* r = (T*)P->d_g;
  T* z = (T*)P->d_t;
  T* q = (T*)P->d_r;
  KParams kp{c.n, 0, tol, 0.0, P->dx * P->dx, P->k00};
  int budget = max_iter;
  for (int attempt = 0; attempt < 3; attempt++) {
    reset_state(P, d);
    CB_HIP(hipMemcpyAsync(P->d_state, P->h_state, sizeof(SolverState), hipMemcpyHostToDevice, c.st));
    hipLaunchKernelGGL(k_zero_off<T>, dim3(c.eblk), dim3(256), 0, c.st, x, S, c.n);
    if (int rc = apply<T>(c, x, u)) return rc;
    hipLaunchKernelGGL(k_mcg_init<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, f, (const T*)u, S, r, z, kp,
                       P->d_state, c.part, c.counter);
    if (int rc = sync_state(P)) return rc;
    if (P->h_state->nonfinite) return CB_E_NONFINITE;
    resid = P->h_state->resid;
    if (P->h_state->done || attempt == 2) return CB_OK;  // true residual checked
    int launched = 0;
    while (launched < budget && !P->h_state->done) {
      const int k = chunk < budget - launched ? chunk : budget - launched;
      for (int i = 0; i < k; i++) {
        if (int rc = apply<T>(c, z, q)) return rc;
        hipLaunchKernelGGL(k_mcg_alpha<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, (const T*)z, (const T*)q, S, kp,
                           P->d_state, c.part, c.counter);
        hipLaunchKernelGGL(k_mcg_update<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, x, r, (const T*)z,
                           (const T*)q, S, kp, P->d_state, c.part, c.counter);
        hipLaunchKernelGGL(k_mcg_dir<T>, dim3(c.eblk), dim3(256), 0, c.st, z, (const T*)r, S, c.n, P->d_state);
      }
      launched += k;
      if (int rc = sync_state(P)) return rc;
      if (P->h_state->nonfinite) return CB_E_NONFINITE;
    }
    iters += P->h_state->iters;
    budget -= launched;
    if (!P->h_state->done) return CB_E_NOCONV;
  }
  return CB_OK;
}

// One adhesive displacement step on state (S in P->d_mask via `S`, p).
// Returns status; fills res (without timing).
template <typename T>
static int adhesive_step(const Ctx& c, const T* f, double d, T* p, unsigned char*& S, unsigned char*& Salt,
                         bool attach_start, double tol, int max_iter, int chunk, double atol, int max_rounds,
                         cb_result* res) {
  cb_plan_s* P = c.P;
  T* u = (T*)P->d_u;
  const double dA = P->dx * P->dx;
  int iters = 0, rounds = 0, status = CB_OK;
  double resid = 0.0;
  if (attach_start) {
    if (int rc = apply<T>(c, p, u)) return rc;
    hipLaunchKernelGGL(k_attach_start<T>, dim3(c.eblk), dim3(256), 0, c.st, f, (const T*)u, d, S, P->d_det, p, c.n);
  } else {
    CB_HIP(hipMemsetAsync(P->d_det, 0, c.n, c.st));
  }
  int* changed = reinterpret_cast<int*>(c.scratch + 8);
  while (rounds < max_rounds) {
    rounds++;
    int rc = set_solve<T>(c, f, d, S, p, tol, max_iter, chunk, iters, resid);
    if (rc != CB_OK) { status = rc; break; }
    if (int e = apply<T>(c, p, u)) return e;
    hipLaunchKernelGGL(k_detach_attach<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, f, (const T*)u, p,
                       (const unsigned char*)S, Salt, P->d_det, P->N, d, P->sigma_c, atol, c.part, c.counter,
                       changed);
    int ch[2];
    CB_HIP(hipMemcpyAsync(ch, changed, sizeof(ch), hipMemcpyDeviceToHost, c.st));
    CB_HIP(hipStreamSynchronize(c.st));
    std::swap(S, Salt);
    if (ch[0] == 0 && ch[1] == 0) break;
    if (rounds == max_rounds) status = CB_E_NOCONV;
  }
  hipLaunchKernelGGL(k_stats<T>, dim3(c.nblk), dim3(RED_THREADS), 0, c.st, (const T*)p, (const T*)u,
                     (const unsigned char*)S, c.n, c.part, c.counter, c.scratch);
  double s4[4];
  if (int rc = read_scratch(c, s4, 4)) return rc;
  res->status = status;
  res->iters = iters;
  res->rounds = rounds;
  res->resid = resid;
  res->F = dA * s4[0];
  res->d = d;
  res->area = dA * s4[1];
  res->U_el = 0.5 * dA * s4[2];
  res->U_ad = -P->dgamma * res->area;
  return status;
}

template <typename T>
static int adhesive_indent(cb_plan_s* P, const T* f, double d, T* p, unsigned char* mask_io,
                           const cb_solve_opts* o, cb_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c = make_ctx(P);
  double tol, atol;
  int max_iter, chunk, init, max_rounds;
  fill_opts(P, o, tol, max_iter, chunk, init, atol, max_rounds);
  *res = cb_result{};
  unsigned char* S = P->d_mask;
  unsigned char* Salt = P->d_mask2;
  hipLaunchKernelGGL(k_mask_overlap<T>, dim3(c.eblk), dim3(256), 0, c.st, f, d, S, p, c.n);
  int rc = adhesive_step<T>(c, f, d, p, S, Salt, false, tol, max_iter, chunk, atol, max_rounds, res);
  if (mask_io && S != mask_io) CB_HIP(hipMemcpyAsync(mask_io, S, c.n, hipMemcpyDeviceToDevice, c.st));
  CB_HIP(hipStreamSynchronize(c.st));
  res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rc != CB_OK) return cb_fail(rc, "adhesive solve did not converge");
  return CB_OK;
}

template <typename T>
static int sweep_impl(cb_plan_s* P, const T* f, const double* dsteps, int nsteps, T* p, unsigned char* mask,
                      const cb_solve_opts* o, cb_result* out) {
  Ctx c = make_ctx(P);
  double tol, atol;
  int max_iter, chunk, init, max_rounds;
  fill_opts(P, o, tol, max_iter, chunk, init, atol, max_rounds);
  unsigned char* S = mask;
  unsigned char* Salt = P->d_mask;
  int first_err = CB_OK;
  for (int k = 0; k < nsteps; k++) {
    const auto t0 = std::chrono::steady_clock::now();
    out[k] = cb_result{};
    int rc = adhesive_step<T>(c, f, dsteps[k], p, S, Salt, true, tol, max_iter, chunk, atol, max_rounds, &out[k]);
    out[k].ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rc != CB_OK && first_err == CB_OK) first_err = rc;
    if (rc == CB_E_DEVICE || rc == CB_E_NONFINITE) break;
  }
  if (S != mask) CB_HIP(hipMemcpyAsync(mask, S, c.n, hipMemcpyDeviceToDevice, c.st));
  CB_HIP(hipStreamSynchronize(c.st));
  if (first_err != CB_OK) return cb_fail(first_err, "a sweep step failed");
  return CB_OK;
}

}  // namespace cb

using namespace cb;

extern "C" int cb_solve_indent(cb_plan P, const void* f, double d, void* p_io, unsigned char* mask_io,
                               const cb_solve_opts* o, cb_result* res) {
  if (!P || !f || !p_io || !res) return cb_fail(CB_E_INVALID, "null argument");
  if (!std::isfinite(d)) return cb_fail(CB_E_INVALID, "d must be finite");
  if (P->dgamma > 0.0) {
    if (P->precision == CB_FP64)
      return adhesive_indent<double>(P, (const double*)f, d, (double*)p_io, mask_io, o, res);
    return adhesive_indent<float>(P, (const float*)f, d, (float*)p_io, mask_io, o, res);
  }
  if (P->precision == CB_FP64)
    return pk_solve<double>(P, (const double*)f, d, false, (double*)p_io, mask_io, o, res);
  return pk_solve<float>(P, (const float*)f, d, false, (float*)p_io, mask_io, o, res);
}

extern "C" int cb_solve_force(cb_plan P, const void* f, double F, void* p_io, unsigned char* mask_io,
                              const cb_solve_opts* o, cb_result* res) {
  if (!P || !f || !p_io || !res) return cb_fail(CB_E_INVALID, "null argument");
  if (!std::isfinite(F) || F < 0.0) return cb_fail(CB_E_INVALID, "F must be finite and >= 0");
  if (P->dgamma > 0.0) return cb_fail(CB_E_UNSUPPORTED, "force control is provided for non-adhesive plans");
  if (P->precision == CB_FP64)
    return pk_solve<double>(P, (const double*)f, F, true, (double*)p_io, mask_io, o, res);
  return pk_solve<float>(P, (const float*)f, F, true, (float*)p_io, mask_io, o, res);
}

extern "C" int cb_sweep(cb_plan P, const void* f, const double* d_steps, int nsteps, void* p_state,
                        unsigned char* mask_state, const cb_solve_opts* o, cb_result* per_step) {
  if (!P || !f || !d_steps || !p_state || !mask_state || !per_step || nsteps < 0)
    return cb_fail(CB_E_INVALID, "null argument or negative step count");
  if (!(P->dgamma > 0.0)) return cb_fail(CB_E_UNSUPPORTED, "sweep needs an adhesive plan (dgamma > 0)");
  for (int k = 0; k < nsteps; k++)
    if (!std::isfinite(d_steps[k])) return cb_fail(CB_E_INVALID, "non-finite displacement step");
  if (P->precision == CB_FP64)
    return sweep_impl<double>(P, (const double*)f, d_steps, nsteps, (double*)p_state, mask_state, o, per_step);
  return sweep_impl<float>(P, (const float*)f, d_steps, nsteps, (float*)p_state, mask_state, o, per_step);
}
