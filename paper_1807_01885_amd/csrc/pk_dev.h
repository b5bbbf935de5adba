// Device helpers shared by the constrained-CG kernels and the row
// transforms that carry part of an iteration's work: block reductions, the
// per-block partial sums, the convergence check and the scalars of the
// search direction.  Inside the iteration the forward row transform (K1)
// forms its own input (the masked gradient, or the search direction, which
// it stores) from arrays already in HBM after folding the partial sums it
// needs, and the inverse row transform (K3) sums the products of its
// output with the contact set's arrays as it writes it (EpiArgs).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace cb {

constexpr int RT = 512;  // threads per solver block (8 waves per CU at 256 blocks)

// Sum / maximum over groups of W lanes (W a power of two up to 64).
template <int W = 64>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W = 64>
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
  return v;
}

// Every thread of an NT-thread block (a power of two) receives the block
// totals (sums, or maxima where mx is set), identical in all threads.
template <int Q, int NT = RT>
__device__ __forceinline__ void block_allreduce(double (&v)[Q], const bool (&mx)[Q]) {
  constexpr int W = NT < 64 ? NT : 64;  // lanes per group
  static_assert(NT > 0 && (NT & (NT - 1)) == 0, "block size must be a power of two");
  __shared__ double sh[NT / W * Q];
  const int lane = threadIdx.x & (W - 1), w = threadIdx.x / W;
#pragma unroll
  for (int q = 0; q < Q; q++) v[q] = mx[q] ? wave_max<W>(v[q]) : wave_sum<W>(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < Q; q++) sh[w * Q + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; q++) {
    double a = sh[q];
    for (int i = 1; i < NT / W; i++) a = mx[q] ? fmax(a, sh[i * Q + q]) : a + sh[i * Q + q];
    v[q] = a;
  }
  __syncthreads();
}

// One Q-tuple of partials per block, after an 8-double header.
template <int Q>
__device__ __forceinline__ void write_partials(double* region, const double (&v)[Q]) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; q++) region[8 + blockIdx.x * Q + q] = v[q];
  }
}

// Totals of the partials of nb blocks, in a fixed order, in every thread.
template <int Q, int NT = RT>
__device__ __forceinline__ void fold(const double* __restrict__ region, int nb, const bool (&mx)[Q],
                                     double (&tot)[Q]) {
#pragma unroll
  for (int q = 0; q < Q; q++) tot[q] = mx[q] ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const double x = region[8 + b * Q + q];
      tot[q] = mx[q] ? fmax(tot[q], x) : tot[q] + x;
    }
  }
  block_allreduce<Q, NT>(tot, mx);
}

__device__ __forceinline__ double* region(double* part, int r) { return part + (size_t)r * REG_STRIDE; }
__device__ __forceinline__ const double* region(const double* part, int r) { return part + (size_t)r * REG_STRIDE; }

// Totals of the gap kernel's partials (S1 = sum g', S2 = sum g'^2, n,
// A1 = sum (s - f), A2 = sum (s - f)^2 over Ic, max(-g') off Ic, a
// non-finite flag): m = mean of g' over Ic under force control (the true
// gap is g' - m), G = sum over Ic of the true gap squared, the relative
// residual, the residual scale, and the stopping test (residual at most
// tol and no cell off Ic penetrating by more than tol x scale).
struct GapTotals {
  double m, G, resid, n, scale;
  bool conv, nonfinite;
};

__device__ __forceinline__ GapTotals gap_totals(const double (&a)[7], const SolverState* st) {
  GapTotals r;
  const bool force = st->force;
  const double nn = a[2];
  r.n = nn;
  r.m = (force && nn > 0.0) ? a[0] / nn : 0.0;
  double G = force ? a[1] - a[0] * r.m : a[1];
  G = G > 0.0 ? G : 0.0;
  r.G = G;
  const double rhs2 = force ? a[4] + 2.0 * r.m * a[3] + nn * r.m * r.m : a[4];
  r.resid = rhs2 > 0.0 ? sqrt(G / rhs2) : sqrt(G);
  const double scale = sqrt((rhs2 > 0.0 ? rhs2 : 0.0) / (nn > 1.0 ? nn : 1.0));
  const double gmin_off = -a[5] - r.m;  // +inf when every cell is in contact
  const bool viol = gmin_off < -st->tol * scale;
  r.nonfinite = a[6] > 0.0;
  r.conv = (r.resid <= st->tol) && !viol;
  r.scale = scale;
  return r;
}

// `writer` records the check; returns true when the solve stops here
__device__ __forceinline__ bool record_check(const GapTotals& gt, SolverState* st, double* gbar2, double s,
                                             int par, bool writer) {
  const bool stop = gt.conv || gt.nonfinite;
  if (writer) {
    st->iters += 1;
    st->resid = gt.resid;
    st->nact = gt.n;
    st->gdev = gt.m;
    st->theta = gt.resid * gt.scale;
    if (st->force) {
      st->d = s + gt.m;
      gbar2[par ^ 1] = s + gt.m;
    }
    if (gt.nonfinite) st->nonfinite = 1;
    if (stop) {
      st->done = 1;
      st->pskip[0] = st->pskip[2] = 1;
    }
  }
  return stop;
}

// The check of an iteration from its gap partials; block 0 records it.
// False when the solve stops here; else gt holds the totals.
template <int NT>
__device__ __forceinline__ bool check_iteration(const EpiArgs& ea, GapTotals& gt) {
  const bool mx7[7] = {false, false, false, false, false, true, true};
  double a[7];
  fold<7, NT>(ea.gap, ea.nb, mx7, a);
  SolverState* st = ea.st;
  const double s = st->force ? ea.gbar2[ea.par] : st->d_in;
  gt = gap_totals(a, st);
  return !record_check(gt, st, ea.gbar2, s, ea.par, blockIdx.x == 0 && threadIdx.x == 0);
}

// Masked gradient of the preconditioned method: the check, then m (and
// G = g.g over Ic, kept for act_scale).  False when the solve stops here.
template <int NT>
__device__ __forceinline__ bool masked_gradient_scalars(const EpiArgs& ea, double& m) {
  GapTotals gt;
  if (!check_iteration<NT>(ea, gt)) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) ea.st->gnorm2 = gt.G;
  m = gt.m;
  return true;
}

// Scalars of the search direction t = Ic ? (x - xbar) + beta t : 0.
// Plain (the check is made here): x = g, xbar = m, beta = G / G_prev.
// Preconditioned (x = z' = M^-1 of the masked gradient): xbar = mean of z'
// over Ic (force control), beta = (g.z') / (g.z')_prev, and act_scale =
// (g.z') / (g.g): a cell that becomes active takes the step
// -tau act_scale g, z' being on a different scale from g (M^-1 damps the
// long waves).  beta = 0 after an update that restarted the directions, and
// (preconditioned) in the first iteration after the switch of
// preconditioner, whose previous sums belong to another one.  False when
// the solve stops here; `pre` tells which x applies.
template <int NT>
__device__ __forceinline__ bool direction_scalars(const EpiArgs& ea, double& xbar, double& beta, bool& pre) {
  SolverState* st = ea.st;
  const bool mx4[4] = {false, false, false, false};
  double u4[4];
  fold<4, NT>(ea.upd, ea.nb, mx4, u4);
  const bool restart = u4[3] != 0.0;
  pre = !(ea.plain0 && (!ea.two || st->phase == 0));
  beta = 0.0;
  if (!pre) {
    GapTotals gt;
    if (!check_iteration<NT>(ea, gt)) return false;
    if (!restart) {
      const bool mx7[7] = {false, false, false, false, false, true, true};
      double b[7];
      fold<7, NT>(ea.gap_prev, ea.nb, mx7, b);
      const double nb2 = b[2];
      const double mb = (st->force && nb2 > 0.0) ? b[0] / nb2 : 0.0;
      const double Gp = st->force ? b[1] - b[0] * mb : b[1];
      beta = Gp > 0.0 ? gt.G / Gp : 0.0;
    }
    xbar = gt.m;
    return true;
  }
  const bool mx2[2] = {false, false};
  double a[2];
  fold<2, NT>(ea.pz, ea.nbz, mx2, a);
  const double nn = st->nact;
  xbar = (st->force && nn > 0.0) ? a[0] / nn : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double G = st->gnorm2;
    st->act_scale = (G > 0.0 && a[1] > 0.0) ? a[1] / G : 1.0;
  }
  if (!restart && st->iters != st->switch_it + 1) {
    double b[2];
    fold<2, NT>(ea.pz_prev, ea.nbz, mx2, b);
    beta = b[1] > 0.0 ? a[1] / b[1] : 0.0;
  }
  return true;
}

}  // namespace cb
