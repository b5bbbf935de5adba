// Iterative contact solves on the device (Sec. 2 after Eq. 11, Eq. 12 and
// the pull-off procedure of Sec. 2).
//
// Non-adhesive: constrained conjugate gradients (Polonsky-Keer reading of
// the paper's reference [8]); the converged pressure solves
//   p >= 0, g = K p + f - d >= 0, p g = 0.
// Optionally the direction is preconditioned by a Fourier multiplier:
// 1/C(kh) = 2/(E1* k K^(k)) (the layered kernel relative to a homogeneous
// one of the coating), which removes the stiffness contrast of thin stiff
// coatings, or 1/K^(k), the inverse of the operator's own symbol, which also
// undoes the 1/k decay of the half-space kernel; the converged pressure is
// the same.
// Adhesive: plain conjugate gradients on the contact set S ((K p)_i = d - f_i
// on S, p = 0 off S), then the Eq. 12 detachment of boundary cells with
// tension above sigma_c and attachment of penetrating cells, repeated until
// nothing changes.
//
// Precision: the solution state (p, u = K p, f, the gap, residuals) is FP64
// in every plan.  The direction vectors (t, K t, M^-1 g, fixed-set CG
// directions) and their convolutions use the plan type TD (FP32 or FP64).
// u is advanced linearly (u -= tau K t) while no cell changes state, and
// recomputed from p by an FP64 convolution whenever a cell is clipped or
// activated and at the end of every chunk, so FP32 direction errors do not
// accumulate in u (iterative refinement inside the iteration).
//
// Reductions: every reduction kernel writes one FP64 partial per block (a
// fixed-order wave/LDS tree); the kernel that needs the total folds the
// partials itself, redundantly in every block and in a fixed order, so all
// blocks hold bitwise-identical scalars and no atomics or grid-wide fences
// are needed.  Scalars that live across iterations are in SolverState;
// those written and read within one iteration are double-buffered by the
// iteration parity.  A chunk of iterations is captured once as a hipGraph
// on the plan's own stream and replayed; the host looks at the convergence
// flag once per chunk.
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"
#include "pk_dev.h"

namespace cb {

#define GRID_LOOP(i, n) for (int i = blockIdx.x * RT + threadIdx.x; i < (n); i += gridDim.x * RT)
// Two consecutive cells per thread and step (n = N^2 is even): 16-byte
// loads of the FP64 arrays, which the widest kernels need to approach the
// bandwidth (the arrays are 16-byte aligned, as the convolution requires).
#define GRID_LOOP2(q, n) for (int q = blockIdx.x * RT + threadIdx.x; q < ((n) >> 1); q += gridDim.x * RT)
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T> using vec2 = typename Vec2<T>::type;

// ---------------------------------------------------------------------------
// Constrained CG (non-adhesive), one iteration =
//   gap
//   [-> z' = M^-1 (Ic (g - m)): K1 checks convergence and forms the masked
//       gradient, K3 sums z' and (g - m) z' over Ic]
//   -> r = K t: K1 forms the direction's scalars (the plain method: after
//      the convergence check) and t, which it stores; K3 sums the step's
//      terms
//   -> update [-> K p]
// (each K1 block folds the partials it needs itself)
// The contact set Ic = {p > 0} is kept as a byte mask `act`, written by the
// update, so that only the update reads p.  Under force control the stored
// p and u lag the true ones by the factor F / (dA sum p) of the previous
// update's sum: every gap block folds that sum and applies the factor as
// it reads u (u recomputed from the stored p scales the same way, K being
// linear), block 0 leaves it in st->pscale for the update, which writes
// true values, and the solve applies the last factor at its end.  The
// recomputation K p after the update runs when a block of the update saw
// a cell change state (it clears st->skip_u, which the gap set).
// ---------------------------------------------------------------------------
// Two-phase solve (two_phase = 1): after QUIET iterations without a change
// of the contact set the direction switches to the inverse-symbol
// preconditioner, which converges fastest on a settled set (one quiet
// iteration measured best: 32.1 mean iterations on the N = 1024 force set
// against 36.4 after two and 37.2 after three).
constexpr int QUIET = 1;
// u = K p is recomputed at least every REFRESH iterations (FP32 linear
// updates drift), whatever the chunking.
constexpr int REFRESH = 16;
// stored gap g' = u + f - s (s = d, or under force control the shift
// gbar[par], the previous mean); partials over Ic = {p > 0}:
// S1 = sum g', S2 = sum g'^2, n, A1 = sum (s - f), A2 = sum (s - f)^2;
// over the rest: max(-g'); and a non-finite flag.
template <typename TD>
__global__ void __launch_bounds__(RT)
k_pk_gap(const unsigned char* __restrict__ act, const double* __restrict__ u, const double* __restrict__ f,
         TD* __restrict__ g, SolverState* __restrict__ st, const double* __restrict__ gbar2,
         double* part, int nb, int n, int par, int two_phase) {
  if (st->done) return;
  const double s = st->force ? gbar2[par] : st->d_in;
  // the previous update's totals: sum p, activations, clips, restarts
  const bool mx4[4] = {false, false, false, false};
  double a4[4];
  fold<4>(region(part, R_UPD), nb, mx4, a4);
  // pending load factor of the stored p and u (force control)
  const double sc = (st->force && a4[0] > 0.0) ? st->Ftarget / (st->dA * a4[0]) : 1.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const bool changed = a4[1] > 0.0 || a4[2] > 0.0;
    st->pscale = sc;
    // u = K p is recomputed after this iteration's update if a cell then
    // changes state (the update clears this) or every REFRESH iterations
    st->skip_u = (st->iters + 1) % REFRESH == 0 ? 0 : 1;
    if (two_phase && st->phase == 0) {
      st->quiet = changed ? 0 : st->quiet + 1;
      if (st->quiet >= QUIET) {
        st->phase = 1;
        st->switch_it = st->iters;
        st->pskip[0] = 1;
        st->pskip[2] = 0;
      }
    }
  }
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY, 0.0};
  const bool mx[7] = {false, false, false, false, false, true, true};
#pragma unroll 2
  GRID_LOOP2(q, n) {
    const double2 f2 = reinterpret_cast<const double2*>(f)[q];
    const double2 u2 = reinterpret_cast<const double2*>(u)[q];
    const uchar2 a2 = reinterpret_cast<const uchar2*>(act)[q];
    const double fv[2] = {f2.x, f2.y}, uv[2] = {u2.x, u2.y};
    const bool av[2] = {a2.x != 0, a2.y != 0};
    TD gv[2];
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const double x = uv[k] * sc + fv[k] - s;
      gv[k] = (TD)x;
      if (!isfinite(x)) v[6] = 1.0;
      if (av[k]) {
        const double a = s - fv[k];
        v[0] += x;
        v[1] += x * x;
        v[2] += 1.0;
        v[3] += a;
        v[4] += a * a;
      } else {
        v[5] = fmax(v[5], -x);
      }
    }
    reinterpret_cast<vec2<TD>*>(g)[q] = vec2<TD>{gv[0], gv[1]};
  }
  block_allreduce<7>(v, mx);
  write_partials<7>(region(part, R_GAP0 + par), v);
}

// tau; p <- max(p - tau t, 0) on Ic; p = 0 and g < -theta -> p = -tau g
// (activation, restarts the conjugate directions); u <- u - tau K t (exact
// while no cell is clipped or activated); partials: sum p, activations,
// clipped cells, activations that restart.  theta = current relative
// residual x rms of (d - f) on Ic: a cell whose penetration is below the
// residual level of the contact set is not activated yet (Polonsky-Keer
// activate at any g < 0, which makes edge cells cycle between clipping and
// activation, each cycle a restart); the stopping test still requires
// g >= -tol x rms everywhere, so the converged solution is the same.
// With `clip` (preconditioned method), a cell clipped in this or the
// previous iteration that re-enters does not restart the directions: such
// bounces at the contact edge otherwise restart nearly every iteration.
template <typename TD>
__global__ void __launch_bounds__(RT)
k_pk_update(double* __restrict__ p, double* __restrict__ u, const TD* __restrict__ g,
            const TD* __restrict__ t, const TD* __restrict__ r, SolverState* __restrict__ st, double* part,
            unsigned char* __restrict__ act, unsigned char* __restrict__ clip, int bounce_from, int nb, int n) {
  if (st->done) return;
  const bool mx4[4] = {false, false, false, false};
  double a[4];
  fold<4>(region(part, R_STEP), nb, mx4, a);
  const double nn = st->nact;
  const double rm = (st->force && nn > 0.0) ? a[2] / nn : 0.0;
  const double rt = a[1] - rm * a[3];
  const double tau = rt > 0.0 ? a[0] / rt : 1.0 / st->k00;
  const double m = st->gdev;
  const double theta = st->theta;
  const double sc = st->pscale;  // pending load factor of the stored p and u
  const bool bounce = clip && st->phase >= bounce_from;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const bool mx[4] = {false, false, false, false};
  const double as = st->act_scale;
#pragma unroll 2
  GRID_LOOP2(q, n) {
    const double2 p2 = reinterpret_cast<const double2*>(p)[q];
    const double2 u2 = reinterpret_cast<const double2*>(u)[q];
    const vec2<TD> t2 = reinterpret_cast<const vec2<TD>*>(t)[q];
    const vec2<TD> g2 = reinterpret_cast<const vec2<TD>*>(g)[q];
    const vec2<TD> r2 = reinterpret_cast<const vec2<TD>*>(r)[q];
    uchar2 c2 = clip ? reinterpret_cast<const uchar2*>(clip)[q] : uchar2{0, 0};
    const double pv[2] = {p2.x, p2.y}, uv[2] = {u2.x, u2.y};
    const double tv[2] = {(double)t2.x, (double)t2.y}, gvv[2] = {(double)g2.x, (double)g2.y};
    const double rv[2] = {(double)r2.x, (double)r2.y};
    const bool cv[2] = {c2.x != 0, c2.y != 0};
    double po[2], uo[2];
    unsigned char ao[2], co[2];
#pragma unroll
    for (int k = 0; k < 2; k++) {
      double pi = pv[k] * sc;
      const bool on = pi > 0.0;
      if (on) pi -= tau * tv[k];
      double pn = pi > 0.0 ? pi : 0.0;
      const bool clipped = on && pn == 0.0;
      if (clipped) v[2] += 1.0;
      const double gi = gvv[k] - m;
      if (pn == 0.0 && gi < -theta) {
        pn = -tau * as * gi;
        v[1] += 1.0;
        if (!bounce || !(clipped || cv[k])) v[3] += 1.0;
      }
      co[k] = clipped ? 1 : 0;
      po[k] = pn;
      ao[k] = pn > 0.0 ? 1 : 0;
      uo[k] = uv[k] * sc - tau * rv[k];
      v[0] += pn;
    }
    if (clip) reinterpret_cast<uchar2*>(clip)[q] = uchar2{co[0], co[1]};
    reinterpret_cast<double2*>(p)[q] = double2{po[0], po[1]};
    reinterpret_cast<uchar2*>(act)[q] = uchar2{ao[0], ao[1]};
    reinterpret_cast<double2*>(u)[q] = double2{uo[0], uo[1]};
  }
  block_allreduce<4>(v, mx);
  write_partials<4>(region(part, R_UPD), v);
  // a cell changed state in this block: u is recomputed from p (every
  // block that writes, writes 0)
  if (threadIdx.x == 0 && (v[1] > 0.0 || v[2] > 0.0)) st->skip_u = 0;
}


// the load factor still pending on the stored p and u when the iterations stop
__global__ void __launch_bounds__(RT) k_pk_pending_scale(double* __restrict__ p, double* __restrict__ u,
                                                         const SolverState* st, int n) {
  const double sc = st->pscale;
  if (sc == 1.0) return;
  GRID_LOOP(i, n) {
    p[i] *= sc;
    u[i] *= sc;
  }
}

// sum p -> R_UPD with the restart flags set (first iteration: no beta)
__global__ void __launch_bounds__(RT) k_pk_seed(const double* __restrict__ p, double* part, int n) {
  const double one = blockIdx.x == 0 && threadIdx.x == 0 ? 1.0 : 0.0;
  double v[4] = {0.0, one, 0.0, one};
  const bool mx[4] = {false, false, false, false};
  GRID_LOOP(i, n) v[0] += p[i];
  block_allreduce<4>(v, mx);
  write_partials<4>(region(part, R_UPD), v);
}

// force control start: p *= F / (dA sum p)
__global__ void __launch_bounds__(RT) k_pk_scale0(double* __restrict__ p, const SolverState* st, const double* part,
                                                  int nb, int n) {
  const bool mx4[4] = {false, false, false, false};
  double a[4];
  fold<4>(region(part, R_UPD), nb, mx4, a);
  if (!(a[0] > 0.0)) return;
  const double sc = st->Ftarget / (st->dA * a[0]);
  GRID_LOOP(i, n) p[i] *= sc;
}

// ---------------------------------------------------------------------------
// Fixed-set CG (adhesive inner solve), one iteration =
//   K z -> zq -> upd -> dir   (x, r in FP64; z, K z in the plan type)
// ---------------------------------------------------------------------------
template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_init(const double* __restrict__ f, const double* __restrict__ u, const unsigned char* __restrict__ S,
           double* __restrict__ r, TD* __restrict__ z, const SolverState* __restrict__ st, double* part, int n) {
  const double d = st->d_in;
  double v[2] = {0.0, 0.0}, w[1] = {0.0};
  const bool mx[2] = {false, true}, mx1[1] = {false};
#pragma unroll 4
  GRID_LOOP(i, n) {
    double ri = 0.0;
    if (S[i]) {
      const double b = d - f[i];
      ri = b - u[i];
      w[0] += b * b;
    }
    r[i] = ri;
    z[i] = (TD)ri;
    v[0] += ri * ri;
    if (!isfinite(ri)) v[1] = 1.0;
  }
  block_allreduce<2>(v, mx);
  write_partials<2>(region(part, R_RR1), v);
  block_allreduce<1>(w, mx1);
  write_partials<1>(region(part, R_INIT), w);
}

__global__ void __launch_bounds__(RT) k_mcg_init_fin(SolverState* st, const double* part, int nb) {
  const bool mx[2] = {false, true}, mx1[1] = {false};
  double a[2], b[1];
  fold<2>(region(part, R_RR1), nb, mx, a);
  fold<1>(region(part, R_INIT), nb, mx1, b);
  if (threadIdx.x == 0) {
    const double bn = sqrt(b[0]);
    st->bnorm = bn;
    st->resid = bn > 0.0 ? sqrt(a[0]) / bn : 0.0;
    if (a[1] > 0.0) { st->nonfinite = 1; st->done = 1; }
    else if (bn == 0.0 || st->resid <= st->tol) st->done = 1;
  }
}

template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_zq(const TD* __restrict__ z, const TD* __restrict__ q, const unsigned char* __restrict__ S,
         const SolverState* __restrict__ st, double* part, int n) {
  if (st->done) return;
  double v[1] = {0.0};
  const bool mx[1] = {false};
#pragma unroll 2
  GRID_LOOP2(k, n) {
    const uchar2 s2 = reinterpret_cast<const uchar2*>(S)[k];
    const vec2<TD> z2 = reinterpret_cast<const vec2<TD>*>(z)[k];
    const vec2<TD> q2 = reinterpret_cast<const vec2<TD>*>(q)[k];
    if (s2.x) v[0] += (double)z2.x * (double)q2.x;
    if (s2.y) v[0] += (double)z2.y * (double)q2.y;
  }
  block_allreduce<1>(v, mx);
  write_partials<1>(region(part, R_ZQ), v);
}

template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_upd(double* __restrict__ x, double* __restrict__ r, const TD* __restrict__ z, const TD* __restrict__ q,
          const unsigned char* __restrict__ S, SolverState* st, double* part, int nb, int n, int par) {
  if (st->done) return;
  const bool mx1[1] = {false}, mx2[2] = {false, true};
  double zq[1], rr[2];
  fold<1>(region(part, R_ZQ), nb, mx1, zq);
  fold<2>(region(part, R_RR0 + (par ^ 1)), nb, mx2, rr);
  if (!(zq[0] > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { st->breakdown = 1; st->done = 1; }
    return;
  }
  const double al = rr[0] / zq[0];
  double v[2] = {0.0, 0.0};
#pragma unroll 4
  GRID_LOOP(i, n) {
    if (S[i]) {
      x[i] += al * (double)z[i];
      const double ri = r[i] - al * (double)q[i];
      r[i] = ri;
      v[0] += ri * ri;
      if (!isfinite(ri)) v[1] = 1.0;
    }
  }
  block_allreduce<2>(v, mx2);
  write_partials<2>(region(part, R_RR0 + par), v);
}

template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_dir(TD* __restrict__ z, const double* __restrict__ r, const unsigned char* __restrict__ S, SolverState* st,
          double* part, int nb, int n, int par) {
  if (st->done) return;
  const bool mx2[2] = {false, true};
  double a[2], b[2];
  fold<2>(region(part, R_RR0 + par), nb, mx2, a);
  fold<2>(region(part, R_RR0 + (par ^ 1)), nb, mx2, b);
  const double bn = st->bnorm;
  const double resid = bn > 0.0 ? sqrt(a[0]) / bn : 0.0;
  const bool stop = a[1] > 0.0 || resid <= st->tol;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iters += 1;
    st->resid = resid;
    if (a[1] > 0.0) st->nonfinite = 1;
    if (stop) st->done = 1;
  }
  if (stop) return;
  const double beta = b[0] > 0.0 ? a[0] / b[0] : 0.0;
#pragma unroll 4
  GRID_LOOP(i, n) z[i] = S[i] ? (TD)(r[i] + beta * (double)z[i]) : TD(0);
}

// Preconditioned fixed-set CG (z = P_S M^-1 P_S r, M^-1 a Fourier multiplier),
// one iteration = K z -> zq -> upd_pc -> M^-1 rt -> ry -> dir_pc.
// start: y = M^-1 r given, rho = r.y over S -> R_RY1, z = S ? y : 0
template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_pc0(const double* __restrict__ r, const TD* __restrict__ y, TD* __restrict__ z,
          const unsigned char* __restrict__ S, const SolverState* __restrict__ st, double* part, int n) {
  if (st->done) return;
  double v[1] = {0.0};
  const bool mx[1] = {false};
#pragma unroll 4
  GRID_LOOP(i, n) {
    const double yi = (double)y[i];
    if (S[i]) v[0] += r[i] * yi;
    z[i] = S[i] ? (TD)yi : TD(0);
  }
  block_allreduce<1>(v, mx);
  write_partials<1>(region(part, R_RY1), v);
}

// alpha = rho / z.q; x += alpha z, r -= alpha q on S; partials |r|^2 (and a
// non-finite flag) -> R_RR[par]; rt = S ? r : 0 in the direction type
template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_upd_pc(double* __restrict__ x, double* __restrict__ r, TD* __restrict__ rt, const TD* __restrict__ z,
             const TD* __restrict__ q, const unsigned char* __restrict__ S, SolverState* st, double* part, int nb,
             int n, int par) {
  if (st->done) return;
  const bool mx1[1] = {false};
  double zq[1], rho[1];
  fold<1>(region(part, R_ZQ), nb, mx1, zq);
  fold<1>(region(part, R_RY0 + (par ^ 1)), nb, mx1, rho);
  if (!(zq[0] > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { st->breakdown = 1; st->done = 1; }
    return;
  }
  const double al = rho[0] / zq[0];
  double v[2] = {0.0, 0.0};
  const bool mx2[2] = {false, true};
#pragma unroll 2
  GRID_LOOP2(k, n) {
    const uchar2 s2 = reinterpret_cast<const uchar2*>(S)[k];
    const vec2<TD> z2 = reinterpret_cast<const vec2<TD>*>(z)[k];
    const vec2<TD> q2 = reinterpret_cast<const vec2<TD>*>(q)[k];
    double2 x2 = reinterpret_cast<const double2*>(x)[k];
    double2 r2 = reinterpret_cast<const double2*>(r)[k];
    double o0 = 0.0, o1 = 0.0;
    if (s2.x) {
      x2.x += al * (double)z2.x;
      o0 = r2.x - al * (double)q2.x;
      r2.x = o0;
      v[0] += o0 * o0;
      if (!isfinite(o0)) v[1] = 1.0;
    }
    if (s2.y) {
      x2.y += al * (double)z2.y;
      o1 = r2.y - al * (double)q2.y;
      r2.y = o1;
      v[0] += o1 * o1;
      if (!isfinite(o1)) v[1] = 1.0;
    }
    reinterpret_cast<double2*>(x)[k] = x2;
    reinterpret_cast<double2*>(r)[k] = r2;
    reinterpret_cast<vec2<TD>*>(rt)[k] = vec2<TD>{(TD)o0, (TD)o1};
  }
  block_allreduce<2>(v, mx2);
  write_partials<2>(region(part, R_RR0 + par), v);
}

// convergence check on |r|; partials r.y over S -> R_RY[par]
template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_ry(const double* __restrict__ r, const TD* __restrict__ y, const unsigned char* __restrict__ S,
         SolverState* st, double* part, int nb, int n, int par) {
  if (st->done) return;
  const bool mx2[2] = {false, true};
  double a[2];
  fold<2>(region(part, R_RR0 + par), nb, mx2, a);
  const double bn = st->bnorm;
  const double resid = bn > 0.0 ? sqrt(a[0]) / bn : 0.0;
  const bool stop = a[1] > 0.0 || resid <= st->tol;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iters += 1;
    st->resid = resid;
    if (a[1] > 0.0) st->nonfinite = 1;
    if (stop) st->done = 1;
  }
  if (stop) return;
  double v[1] = {0.0};
  const bool mx[1] = {false};
#pragma unroll 2
  GRID_LOOP2(k, n) {
    const uchar2 s2 = reinterpret_cast<const uchar2*>(S)[k];
    const double2 r2 = reinterpret_cast<const double2*>(r)[k];
    const vec2<TD> y2 = reinterpret_cast<const vec2<TD>*>(y)[k];
    if (s2.x) v[0] += r2.x * (double)y2.x;
    if (s2.y) v[0] += r2.y * (double)y2.y;
  }
  block_allreduce<1>(v, mx);
  write_partials<1>(region(part, R_RY0 + par), v);
}

// z = S ? y + beta z : 0, beta = rho_new / rho_old
template <typename TD>
__global__ void __launch_bounds__(RT)
k_mcg_dir_pc(TD* __restrict__ z, const TD* __restrict__ y, const unsigned char* __restrict__ S,
             const SolverState* __restrict__ st, double* part, int nb, int n, int par) {
  if (st->done) return;
  const bool mx1[1] = {false};
  double a[1], b[1];
  fold<1>(region(part, R_RY0 + par), nb, mx1, a);
  fold<1>(region(part, R_RY0 + (par ^ 1)), nb, mx1, b);
  const double beta = b[0] > 0.0 ? a[0] / b[0] : 0.0;
#pragma unroll 2
  GRID_LOOP2(k, n) {
    const uchar2 s2 = reinterpret_cast<const uchar2*>(S)[k];
    const vec2<TD> y2 = reinterpret_cast<const vec2<TD>*>(y)[k];
    const vec2<TD> z2 = reinterpret_cast<const vec2<TD>*>(z)[k];
    reinterpret_cast<vec2<TD>*>(z)[k] = vec2<TD>{s2.x ? (TD)((double)y2.x + beta * (double)z2.x) : TD(0),
                                                 s2.y ? (TD)((double)y2.y + beta * (double)z2.y) : TD(0)};
  }
}

// ---------------------------------------------------------------------------
// small kernels: initial guesses, masks, statistics
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(RT) k_init_disp(double* __restrict__ p, const double* __restrict__ f, int n,
                                                  double d, double k00) {
  GRID_LOOP(i, n) {
    const double v = d - f[i];
    p[i] = v > 0.0 ? v / k00 : 0.0;
  }
}
__global__ void __launch_bounds__(RT) k_fill(double* __restrict__ p, int n, double v) { GRID_LOOP(i, n) p[i] = v; }
__global__ void __launch_bounds__(RT) k_clamp_pos(double* __restrict__ p, int n) {
  GRID_LOOP(i, n) p[i] = p[i] > 0.0 ? p[i] : 0.0;
}
__global__ void __launch_bounds__(RT) k_mask_from_p(const double* __restrict__ p, unsigned char* __restrict__ S,
                                                    int n) {
  GRID_LOOP(i, n) S[i] = p[i] > 0.0 ? 1 : 0;
}
__global__ void __launch_bounds__(RT) k_zero_off(double* __restrict__ p, const unsigned char* __restrict__ S,
                                                 int n) {
  GRID_LOOP(i, n) if (!S[i]) p[i] = 0.0;
}
__global__ void __launch_bounds__(RT) k_zero_bytes(unsigned char* __restrict__ a, int n) { GRID_LOOP(i, n) a[i] = 0; }

// min f, max f, non-finite -> R_MISC (as max of -f, max of f, flag)
// -min f, max f, non-finite flag, and max p of a caller's guess (p nullable)
__global__ void __launch_bounds__(RT) k_minmax(const double* __restrict__ x, const double* __restrict__ p,
                                               double* part, int n) {
  double v[4] = {-INFINITY, -INFINITY, 0.0, -INFINITY};
  const bool mx[4] = {true, true, true, true};
  GRID_LOOP(i, n) {
    const double a = x[i];
    v[0] = fmax(v[0], -a);
    v[1] = fmax(v[1], a);
    if (!isfinite(a)) v[2] = 1.0;
    if (p) v[3] = fmax(v[3], p[i]);
  }
  block_allreduce<4>(v, mx);
  write_partials<4>(region(part, R_MISC), v);
}

// Histogram of the profile depth e = f - fmin for the force-control cold
// start: HB bins, bin 0 e <= emin, bin b e in (emin r^(b-1), emin r^b];
// per block the cell counts and the sums of e in fixed point (units of
// range 2^-40, so that the totals are exact and order-independent), into
// out[block][2 HB].
constexpr int HB = 128;
constexpr double HSPAN = 1e7;  // emin = range / HSPAN
__global__ void __launch_bounds__(RT) k_depth_hist(const double* __restrict__ f, double fmin, double range,
                                                   unsigned long long* __restrict__ out, int n) {
  __shared__ unsigned long long h[2 * HB];
  for (int i = threadIdx.x; i < 2 * HB; i += RT) h[i] = 0ull;
  __syncthreads();
  const double emin = range / HSPAN;
  const double inv_lr = (HB - 1) / log(HSPAN);
  const double unit = 1099511627776.0 / range;  // 2^40 / range
  GRID_LOOP(i, n) {
    const double e = f[i] - fmin;
    int b = e > emin ? 1 + (int)(log(e / emin) * inv_lr) : 0;
    b = b < HB - 1 ? b : HB - 1;
    const double q = e * unit + 0.5;
    atomicAdd(&h[b], 1ull);
    atomicAdd(&h[HB + b], (unsigned long long)(q > 0.0 ? q : 0.0));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * HB; i += RT) out[(size_t)blockIdx.x * 2 * HB + i] = h[i];
}
// Sum of the block histograms as doubles: counts, then sums of e in units
// of range 2^-40.  The sums are integers, exact in any order: each thread
// takes every G-th block histogram with eight loads in flight (one load
// per round trip took 62 us at 256 blocks), and the G group totals meet
// in LDS.
__global__ void __launch_bounds__(RT) k_depth_hist_fold(const unsigned long long* __restrict__ in, int nb,
                                                        double* __restrict__ out) {
  constexpr int W = 2 * HB, G = RT / W;
  static_assert(RT % W == 0, "block must hold whole histograms");
  __shared__ unsigned long long part[G][W];
  const int i = threadIdx.x % W, g = threadIdx.x / W;
  unsigned long long t[8] = {};
  int b = g;
  for (; b + 7 * G < nb; b += 8 * G) {
#pragma unroll
    for (int k = 0; k < 8; k++) t[k] += in[(size_t)(b + k * G) * W + i];
  }
  for (; b < nb; b += G) t[0] += in[(size_t)b * W + i];
  unsigned long long s = 0ull;
#pragma unroll
  for (int k = 0; k < 8; k++) s += t[k];
  part[g][i] = s;
  __syncthreads();
  if (g == 0) {
    for (int q = 1; q < G; q++) s += part[q][i];
    out[i] = (double)s;
  }
}

// sum p, |S| (or |p > 0|), sum p u, non-finite -> R_MISC
__global__ void __launch_bounds__(RT)
k_stats(const double* __restrict__ p, const double* __restrict__ u, const unsigned char* __restrict__ S, double* part,
        int n) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const bool mx[4] = {false, false, false, true};
  GRID_LOOP(i, n) {
    const double pi = p[i];
    v[0] += pi;
    v[1] += S ? (S[i] ? 1.0 : 0.0) : (pi > 0.0 ? 1.0 : 0.0);
    v[2] += pi * u[i];
    if (!isfinite(pi)) v[3] = 1.0;
  }
  block_allreduce<4>(v, mx);
  write_partials<4>(region(part, R_MISC), v);
}

// fold R_MISC (Q quantities, max-mask bits) into the scratch area
template <int Q>
__global__ void __launch_bounds__(RT) k_fold_misc(double* part, int nb, int maxmask) {
  bool mx[Q];
#pragma unroll
  for (int q = 0; q < Q; q++) mx[q] = (maxmask >> q) & 1;
  double tot[Q];
#pragma unroll
  for (int q = 0; q < Q; q++) tot[q] = mx[q] ? -INFINITY : 0.0;
  const double* reg = region(part, R_MISC);
  for (int b = threadIdx.x; b < nb; b += RT) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const double x = reg[8 + b * Q + q];
      tot[q] = mx[q] ? fmax(tot[q], x) : tot[q] + x;
    }
  }
  __shared__ double sh[RT / 64 * Q];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; q++) tot[q] = mx[q] ? wave_max(tot[q]) : wave_sum(tot[q]);
  if (lane == 0)
    for (int q = 0; q < Q; q++) sh[w * Q + q] = tot[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < Q; q++) {
      double a = sh[q];
      for (int i = 1; i < RT / 64; i++) a = mx[q] ? fmax(a, sh[i * Q + q]) : a + sh[i * Q + q];
      part[SCRATCH_OFF + q] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// Adhesive kernels
// ---------------------------------------------------------------------------
// S0 = {f - d <= 0}, p = 0, no cell detached yet
__global__ void __launch_bounds__(RT)
k_mask_overlap(const double* __restrict__ f, double d, unsigned char* __restrict__ S, unsigned char* __restrict__ det,
               double* __restrict__ p, int n) {
  GRID_LOOP(i, n) {
    S[i] = (f[i] - d <= 0.0) ? 1 : 0;
    det[i] = 0;
    p[i] = 0.0;
  }
}

// Start of a displacement step: S |= {f - d + u < 0}, p = 0 off S, det = 0
__global__ void __launch_bounds__(RT)
k_attach_start(const double* __restrict__ f, const double* __restrict__ u, double d, unsigned char* __restrict__ S,
               unsigned char* __restrict__ det, double* __restrict__ p, int n) {
  GRID_LOOP(i, n) {
    const bool s = S[i] || (f[i] - d + u[i] < 0.0);
    S[i] = s ? 1 : 0;
    det[i] = 0;
    if (!s) p[i] = 0.0;
  }
}

// Eq. 12 detachment of boundary cells (a 4-neighbour outside S, or on the
// grid edge) with p < -sigma_c, attachment of cells outside S with
// f - d + u < -atol that were not detached in this step.  Reads Sin,
// writes Sout; partials (detached, attached) -> R_MISC.
__global__ void __launch_bounds__(RT)
k_detach_attach(const double* __restrict__ f, const double* __restrict__ u, double* __restrict__ p,
                const unsigned char* __restrict__ Sin, unsigned char* __restrict__ Sout,
                unsigned char* __restrict__ det, int N, double d, double sigma_c, double atol, double* part) {
  const int n = N * N;
  double v[2] = {0.0, 0.0};
  const bool mx[2] = {false, false};
  GRID_LOOP(i, n) {
    const int r = i / N, c = i - r * N;
    const bool s = Sin[i] != 0;
    bool ns = s;
    if (s) {
      const bool inner = r > 0 && r < N - 1 && c > 0 && c < N - 1 && Sin[i - 1] && Sin[i + 1] &&
                         Sin[i - N] && Sin[i + N];
      if (!inner && p[i] < -sigma_c) {
        ns = false;
        det[i] = 1;
        p[i] = 0.0;
        v[0] += 1.0;
      }
    } else if (!det[i] && (f[i] - d + u[i] < -atol)) {
      ns = true;
      v[1] += 1.0;
    }
    Sout[i] = ns ? 1 : 0;
  }
  block_allreduce<2>(v, mx);
  write_partials<2>(region(part, R_MISC), v);
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
struct Ctx {
  cb_plan_s* P;
  hipStream_t st;   // the plan's own stream
  int n, nb;
};

static Ctx make_ctx(cb_plan_s* P) {
  Ctx c;
  c.P = P;
  c.st = P->istream;
  c.n = P->N * P->N;
  c.nb = P->nbr;
  return c;
}

// Order the plan stream after the caller's stream.
static int enter(cb_plan_s* P) {
  CB_HIP(hipEventRecord(P->ev_in, P->stream));
  CB_HIP(hipStreamWaitEvent(P->istream, P->ev_in, 0));
  return CB_OK;
}

static int read_scratch(const Ctx& c, double* out, int k) {
  CB_HIP(hipMemcpyAsync(out, c.P->d_part + SCRATCH_OFF, k * sizeof(double), hipMemcpyDeviceToHost, c.st));
  CB_HIP(hipStreamSynchronize(c.st));
  return CB_OK;
}

static int read_state(cb_plan_s* P, SolverState* out) {
  CB_HIP(hipMemcpyAsync(P->h_state, P->d_state, sizeof(SolverState), hipMemcpyDeviceToHost, P->istream));
  CB_HIP(hipStreamSynchronize(P->istream));
  *out = *P->h_state;
  return CB_OK;
}

static int write_state(cb_plan_s* P, const SolverState& s) {
  P->h_state[0] = s;
  CB_HIP(hipMemcpyAsync(P->d_state, P->h_state, sizeof(SolverState), hipMemcpyHostToDevice, P->istream));
  return CB_OK;
}

// direction-type convolution (plan precision), optionally with another table
static hipError_t apply_dir(const Ctx& c, const void* x, void* y, const int* skip, const void* table = nullptr,
                            const EpiArgs* epi = nullptr) {
  return launch_apply(c.P, x, y, c.st, 7, skip, table, -1, epi);
}
// Fourier preconditioner (N-periodic convolution with the symbol `table`)
static hipError_t apply_pc(const Ctx& c, const void* x, void* y, const int* skip, const void* table,
                           const EpiArgs* epi = nullptr) {
  return launch_apply(c.P, x, y, c.st, 15, skip, table, -1, epi);
}
// FP64 convolution of the FP64 state
static hipError_t apply64(const Ctx& c, const double* x, double* y, const int* skip) {
  return launch_apply(c.P, x, y, c.st, 7, skip, nullptr, 0);
}

// gbar double buffer lives in the scratch tail (2 doubles)
static double* gbar2_ptr(cb_plan_s* P) { return P->d_part + SCRATCH_OFF + 24; }

template <typename TD>
// pk: 0 plain, 1 preconditioned by 1/C(kh), 2 preconditioned by 1/K^
// mode: 0 plain, 1 / 2 preconditioned by 1/C(kh) / 1/K^ throughout; 3 / 4
// two-phase, plain / 1/C(kh) until the contact set settles, then 1/K^.
// second: a two-phase solve already past its switch (the host saw phase 1):
// the first phase's block, which would only exit at entry, is left out.
static hipError_t pk_enqueue_chunk(const Ctx& c, double* p, const double* f, bool force, int mode, int chunk,
                                   bool second = false) {
  cb_plan_s* P = c.P;
  const bool two = mode >= 3;
  const int pk0 = two ? mode - 3 : mode;  // preconditioner of the first (or only) phase
  double* u = (double*)P->d_u;
  TD* g = (TD*)P->d_g;  // the gap in the direction type (FP32 plans: FP32)
  unsigned char* act = P->d_mask2;  // contact set {p > 0}
  TD* t = (TD*)P->d_t;
  TD* r = (TD*)P->d_r;
  SolverState* st = P->d_state;
  double* part = P->d_part;
  double* gb = gbar2_ptr(P);
  const dim3 grid(c.nb), blk(RT);
  const int* skip_done = &st->done;   // {done, zero}
  const int* skip_u = &st->skip_u;    // {skip_u, done}
  // blocks of the inverse row transforms that carry the step and z' sums
  const int nb3d = rows_blocks(P, -1, P->kernel_mode == CB_KERNEL_PERIODIC), nb3p = rows_blocks(P, -1, true);
  // the fused row-transform sums write 4 (step) or 2 (z') partials per block
  if (nb3d < 1 || nb3p < 1 || 4 * nb3d > REG_STRIDE - 8 || 2 * nb3p > REG_STRIDE - 8) return hipErrorInvalidValue;
  double* pgap = part + (size_t)(R_GAP0) * REG_STRIDE;
  double* ppz = part + (size_t)(R_PZ0) * REG_STRIDE;
  // The preconditioned gradient of one phase (none for the plain method):
  // the periodic convolution's forward row transform checks convergence and
  // forms the masked gradient from g, z' = M^-1 of it goes into r (free
  // until K t is formed), its inverse row transform sums z' and (g - m) z'
  // over the contact set.
  auto precondition = [&](int pc_k, const int* skip, int par) -> hipError_t {
    if (pc_k == 0) return hipSuccess;
    EpiArgs ez;
    ez.mode = 2;
    ez.pro = 1;
    ez.act = act;
    ez.g = g;
    ez.st = st;
    ez.region = ppz + (size_t)par * REG_STRIDE;
    ez.gap = pgap + (size_t)par * REG_STRIDE;
    ez.gbar2 = gb;
    ez.nb = c.nb;
    ez.par = par;
    return apply_pc(c, g, r, skip, pc_k == 2 ? P->d_pinv : P->d_ptable, &ez);
  };
  for (int i = 0; i < chunk; i++) {
    const int par = i & 1;
    hipLaunchKernelGGL(k_pk_gap<TD>, grid, blk, 0, c.st, (const unsigned char*)act, (const double*)u, f, g, st, gb,
                       part, c.nb, c.n, par, two ? 1 : 0);
    if (two) {
      if (!second)
        if (hipError_t e = precondition(pk0, &st->pskip[0], par)) return e;
      if (hipError_t e = precondition(2, &st->pskip[2], par)) return e;
    } else if (hipError_t e = precondition(pk0, skip_done, par)) {
      return e;
    }
    // the forward row transform forms the direction (plain, or from z' in r)
    // and stores t; r = K t; the inverse row transform forms the step's sums
    EpiArgs es;
    es.mode = 1;
    es.pro = 2;
    es.act = act;
    es.g = g;
    es.t = t;
    es.st = st;
    es.region = part + (size_t)R_STEP * REG_STRIDE;
    es.x = r;
    es.tdir = t;
    es.gap = pgap + (size_t)par * REG_STRIDE;
    es.gap_prev = pgap + (size_t)(par ^ 1) * REG_STRIDE;
    es.pz = ppz + (size_t)par * REG_STRIDE;
    es.pz_prev = ppz + (size_t)(par ^ 1) * REG_STRIDE;
    es.upd = part + (size_t)R_UPD * REG_STRIDE;
    es.gbar2 = gb;
    es.nb = c.nb;
    es.nbz = nb3p;
    es.par = par;
    es.plain0 = pk0 == 0 ? 1 : 0;
    es.two = two ? 1 : 0;
    if (hipError_t e = apply_dir(c, t, r, skip_done, nullptr, &es)) return e;
    // the bounce rule of the preconditioned directions (from phase 0 when
    // that phase is preconditioned, else from the switch)
    const bool clip = two || pk0 > 0;
    hipLaunchKernelGGL(k_pk_update<TD>, grid, blk, 0, c.st, p, u, (const TD*)g, (const TD*)t, (const TD*)r, st, part,
                       act, clip ? P->d_det : nullptr, pk0 > 0 ? 0 : 1, nb3d, c.n);
    if (hipError_t e = apply64(c, p, u, skip_u)) return e;
  }
  return hipGetLastError();
}

template <typename TD>
// pk: 0 plain CG, 1 / 2 preconditioned by 1/C(kh) / 1/K^
static hipError_t mcg_enqueue_chunk(const Ctx& c, double* x, const unsigned char* S, int chunk, int pk) {
  cb_plan_s* P = c.P;
  double* r = (double*)P->d_g;
  TD* z = (TD*)P->d_t;
  TD* q = (TD*)P->d_r;
  SolverState* st = P->d_state;
  double* part = P->d_part;
  const dim3 grid(c.nb), blk(RT);
  if (pk > 0) {
    TD* rt = (TD*)P->d_pold;
    TD* y = (TD*)P->d_y;
    const void* ptab = pk == 2 ? P->d_pinv : P->d_ptable;
    for (int i = 0; i < chunk; i++) {
      const int par = i & 1;
      if (hipError_t e = apply_dir(c, z, q, &st->done)) return e;
      hipLaunchKernelGGL(k_mcg_zq<TD>, grid, blk, 0, c.st, (const TD*)z, (const TD*)q, S, st, part, c.n);
      hipLaunchKernelGGL(k_mcg_upd_pc<TD>, grid, blk, 0, c.st, x, r, rt, (const TD*)z, (const TD*)q, S, st, part,
                         c.nb, c.n, par);
      if (hipError_t e = apply_pc(c, rt, y, &st->done, ptab)) return e;
      hipLaunchKernelGGL(k_mcg_ry<TD>, grid, blk, 0, c.st, (const double*)r, (const TD*)y, S, st, part, c.nb, c.n,
                         par);
      hipLaunchKernelGGL(k_mcg_dir_pc<TD>, grid, blk, 0, c.st, z, (const TD*)y, S, st, part, c.nb, c.n, par);
    }
    return hipGetLastError();
  }
  for (int i = 0; i < chunk; i++) {
    const int par = i & 1;
    if (hipError_t e = apply_dir(c, z, q, &st->done)) return e;
    hipLaunchKernelGGL(k_mcg_zq<TD>, grid, blk, 0, c.st, (const TD*)z, (const TD*)q, S, st, part, c.n);
    hipLaunchKernelGGL(k_mcg_upd<TD>, grid, blk, 0, c.st, x, r, (const TD*)z, (const TD*)q, S, st, part, c.nb, c.n,
                       par);
    hipLaunchKernelGGL(k_mcg_dir<TD>, grid, blk, 0, c.st, z, (const double*)r, S, st, part, c.nb, c.n, par);
  }
  return hipGetLastError();
}

// Captured graph of one chunk, cached per (kind, pointers, chunk).
template <class Enq>
static hipGraphExec_t chunk_graph(cb_plan_s* P, int kind, const void* a, const void* b, const void* cc, int chunk,
                                  Enq enqueue) {
  if (!P->use_graphs) return nullptr;
  GraphEntry* lru = &P->graphs[0];
  for (auto& e : P->graphs) {
    if (e.exec && e.kind == kind && e.a == a && e.b == b && e.c == cc && e.chunk == chunk) {
      e.used = ++P->graph_clock;
      return e.exec;
    }
    if (!e.exec || e.used < lru->used) lru = &e;
  }
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  // the stream's earlier work (on this plan's stream only) has completed
  // when a chunk is captured: run_chunks waits for every chunk it launches
  std::lock_guard<std::mutex> lk(graph_mutex());
  if (hipStreamBeginCapture(P->istream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    P->use_graphs = 0;
    (void)hipGetLastError();
    return nullptr;
  }
  const hipError_t e1 = enqueue();
  const hipError_t e2 = hipStreamEndCapture(P->istream, &g);
  if (e1 != hipSuccess || e2 != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    P->use_graphs = 0;
    (void)hipGetLastError();
    return nullptr;
  }
  (void)hipGraphDestroy(g);
  if (lru->exec) {
    // an evicted executable graph is kept until the plan is destroyed; a
    // long list is released once the plan's stream has drained
    P->retired.push_back(lru->exec);
    if (P->retired.size() > 64 && hipStreamSynchronize(P->istream) == hipSuccess) {
      for (hipGraphExec_t r : P->retired) (void)hipGraphExecDestroy(r);
      P->retired.clear();
    }
  }
  lru->kind = kind;
  lru->a = a;
  lru->b = b;
  lru->c = cc;
  lru->chunk = chunk;
  lru->exec = ex;
  lru->used = ++P->graph_clock;
  return ex;
}

// Run chunks until the device flags convergence (or max_iter launched).
// One chunk is in flight at a time: its iterations after convergence exit
// at entry but still cost a dispatch each (about 25 us of GPU time per
// iteration at N = 1024, and in a concurrent batch they hold the hardware
// queues they share with other solves), so the length of the next chunk
// follows the residual's progress: the iterations still needed at the
// rate of the last chunk (from r0 at iteration 0 for the first), rounded
// up to a power of two in [2, chunk].  The first chunk is min(8, chunk).
// A solve whose state reaches phase 1 continues with kind1 / enqueue1
// (the same iteration without its first phase's kernels).
template <class Enq, class Enq1>
static int run_chunks(cb_plan_s* P, int kind, int kind1, const void* a, const void* b, const void* cc, int chunk,
                      int max_iter, Enq enqueue, Enq1 enqueue1, SolverState* out, double r0) {
  int launched = 0, len = chunk < 8 ? chunk : 8;
  double r_prev = r0;
  int it_prev = 0;
  bool second = false;
  while (true) {
    const int n = len;
    hipGraphExec_t ex = second ? chunk_graph(P, kind1, a, b, cc, n, [&]() { return enqueue1(n); })
                               : chunk_graph(P, kind, a, b, cc, n, [&]() { return enqueue(n); });
    if (ex) CB_HIP(hipGraphLaunch(ex, P->istream));
    else CB_HIP(second ? enqueue1(n) : enqueue(n));
    launched += n;
    CB_HIP(hipMemcpyAsync(&P->h_state[0], P->d_state, sizeof(SolverState), hipMemcpyDeviceToHost, P->istream));
    CB_HIP(hipEventRecord(P->ev_state[0], P->istream));
    CB_HIP(hipEventSynchronize(P->ev_state[0]));
    const SolverState& s = P->h_state[0];
    if (s.done || s.nonfinite || launched >= max_iter) break;
    second = second || s.phase == 1;
    len = chunk;
    if (r_prev > 0.0 && s.resid > 0.0 && s.resid < r_prev && s.iters > it_prev && s.tol > 0.0) {
      const double rate = (std::log(s.resid) - std::log(r_prev)) / (s.iters - it_prev);  // < 0
      const double need = (std::log(s.tol) - std::log(s.resid)) / rate + 1.0;
      len = 2;
      while (len < chunk && len < need) len *= 2;
      if (len > chunk) len = chunk;
    }
    r_prev = s.resid;
    it_prev = s.iters;
  }
  CB_HIP(hipStreamSynchronize(P->istream));
  return read_state(P, out);
}

struct Opts {
  double tol, atol, preload_d;
  int max_iter, chunk, init, max_rounds, precond;
};

static Opts fill_opts(const cb_plan_s* P, const cb_solve_opts* o) {
  cb_solve_opts d{};
  d.precond = -1;
  d.attach_tol = -1.0;
  d.preload_d = -HUGE_VAL;
  if (o) d = *o;
  Opts r;
  r.tol = d.tol > 0 ? d.tol : (P->precision == CB_FP64 ? 1e-10 : 1e-8);
  r.max_iter = d.max_iter > 0 ? d.max_iter : 20000;
  r.chunk = d.chunk > 0 ? d.chunk : 16;
  r.chunk += r.chunk & 1;  // even: iteration parity restarts at 0 in every chunk
  if (r.chunk > r.max_iter) r.chunk = r.max_iter + (r.max_iter & 1);
  r.init = d.init;
  r.atol = d.attach_tol >= 0 ? d.attach_tol : (P->precision == CB_FP64 ? 1e-12 : 1e-9) * P->L;
  r.max_rounds = d.max_rounds > 0 ? d.max_rounds : 10000;
  r.precond = d.precond;
  r.preload_d = d.preload_d;
  return r;
}

static SolverState base_state(const cb_plan_s* P, double tol, double d_in, bool force, double F) {
  SolverState s{};
  s.tol = tol;
  s.Ftarget = F;
  s.dA = P->dx * P->dx;
  s.k00 = P->k00;
  s.d_in = d_in;
  s.force = force ? 1 : 0;
  s.d = d_in;
  s.act_scale = 1.0;
  s.pscale = 1.0;
  s.switch_it = -2;
  s.pskip[2] = 1;  // the phase-1 block idles until the switch
  return s;
}

// Force-control cold start: the overlap {f < d0} of the rigid indenter at
// an approach d0 estimated from the distribution of the profile depth
// e = f - fmin, with p0 = d0 - f there (the solve rescales it to F).  A
// region of area A pressed to mean depth dbar carries about
// 1.1 E(k) sqrt(A) dbar, with E(k) = E1* / C(k h) the layered modulus at
// k = 2 / sqrt(A) (on a half-space the exact factors are 2/sqrt(pi) = 1.13
// for a flat punch, 1.06 for a paraboloid, about 1.1 for a cone).  d0 is
// taken at 0.7
// of the depth where that force reaches F, since the overlap exceeds the
// contact of curved indenters.  A uniform start over the grid spends most
// of its iterations shrinking the contact set (CPU sweep of the N = 256
// force set: 670 -> 473 iterations).  Too large a load for any overlap:
// the uniform start.
static int cold_start_force(const Ctx& c, const double* f, double fmin, double fmax, double F, double* p,
                            bool* found_out) {
  cb_plan_s* P = c.P;
  const dim3 grid(c.nb), blk(RT);
  const double range = fmax - fmin;
  double d0 = 0.0;
  bool found = false;
  if (range > 0.0) {
    // block histograms in y (2 HB words each; N^2 >= 2 HB words for N >= 16)
    int nbh = (int)std::min<long long>(c.nb, std::max<long long>(1, (long long)c.n / (2 * HB)));
    hipLaunchKernelGGL(k_depth_hist, dim3(nbh), blk, 0, c.st, f, fmin, range, (unsigned long long*)P->d_y, c.n);
    hipLaunchKernelGGL(k_depth_hist_fold, dim3(1), blk, 0, c.st, (const unsigned long long*)P->d_y, nbh,
                       (double*)P->d_pold);
    double hist[2 * HB];
    CB_HIP(hipMemcpyAsync(hist, P->d_pold, sizeof(hist), hipMemcpyDeviceToHost, c.st));
    CB_HIP(hipStreamSynchronize(c.st));
    const double emin = range / HSPAN, r = std::pow(HSPAN, 1.0 / (HB - 1));
    const double unit = range / 1099511627776.0;
    const double dA = P->dx * P->dx;
    double C = 0.0, S = 0.0, edge = emin;
    for (int b = 0; b < HB && !found; b++, edge *= r) {
      C += hist[b];
      S += hist[HB + b] * unit;
      if (C <= 0.0) continue;
      const double A = C * dA, dbar = edge - S / C, k = 2.0 / std::sqrt(A);
      const double Fm = 1.1 * P->E1s / plan_shape(P, k) * std::sqrt(A) * dbar;
      if (Fm >= F) {
        d0 = fmin + 0.7 * edge;
        found = true;
      }
    }
  }
  *found_out = found;
  if (found) hipLaunchKernelGGL(k_init_disp, grid, blk, 0, c.st, p, f, c.n, d0, P->k00);
  else hipLaunchKernelGGL(k_fill, grid, blk, 0, c.st, p, c.n, F / (P->dx * P->dx * c.n));
  CB_HIP(hipGetLastError());
  return CB_OK;
}

template <typename TD>
static int pk_solve(cb_plan_s* P, const double* f, double target, bool force, double* p, unsigned char* mask,
                    const cb_solve_opts* o, cb_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c = make_ctx(P);
  const Opts op = fill_opts(P, o);
  const double dA = P->dx * P->dx;
  *res = cb_result{};
  if (op.precond < -1 || op.precond > 3) return cb_fail(CB_E_INVALID, "precond must be -1, 0, 1, 2 or 3");
  if (int rc = enter(P)) return rc;
  const dim3 grid(c.nb), blk(RT);
  hipLaunchKernelGGL(k_minmax, grid, blk, 0, c.st, f, op.init == 1 ? (const double*)p : nullptr, P->d_part, c.n);
  hipLaunchKernelGGL(k_fold_misc<4>, dim3(1), blk, 0, c.st, P->d_part, c.nb, 15);
  double mm[4];
  if (int rc = read_scratch(c, mm, 4)) return rc;
  if (mm[2] > 0.0) return cb_fail(CB_E_NONFINITE, "profile f contains NaN/Inf");
  const double fmin = -mm[0], fmax = mm[1];
  // a caller's guess without a positive value is no guess: cold start
  const bool guess = op.init == 1 && mm[3] > 0.0;
  const bool trivial = force ? !(target > 0.0) : (target <= fmin);
  if (trivial) {
    hipLaunchKernelGGL(k_fill, grid, blk, 0, c.st, p, c.n, 0.0);
    if (mask) hipLaunchKernelGGL(k_zero_bytes, grid, blk, 0, c.st, mask, c.n);
    CB_HIP(hipStreamSynchronize(c.st));
    res->status = CB_OK;
    res->d = force ? fmin : target;
    res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return CB_OK;
  }
  // initial pressure; `near`: a start whose support is close to the contact
  bool near = guess;
  if (guess) {
    hipLaunchKernelGGL(k_clamp_pos, grid, blk, 0, c.st, p, c.n);
  } else if (force) {
    if (int rc = cold_start_force(c, f, fmin, fmax, target, p, &near)) return rc;
  } else {
    hipLaunchKernelGGL(k_init_disp, grid, blk, 0, c.st, p, f, c.n, target, P->k00);
  }
  if (int rc = write_state(P, base_state(P, op.tol, force ? 0.0 : target, force, force ? target : 0.0))) return rc;
  CB_HIP(hipMemsetAsync(gbar2_ptr(P), 0, 2 * sizeof(double), c.st));
  // direction buffers start at zero so that a solve never depends on what a
  // previous call left in the workspace
  CB_HIP(hipMemsetAsync(P->d_t, 0, (size_t)c.n * 8, c.st));
  CB_HIP(hipMemsetAsync(P->d_r, 0, (size_t)c.n * 8, c.st));
  CB_HIP(hipMemsetAsync(P->d_pold, 0, (size_t)c.n * 8, c.st));
  hipLaunchKernelGGL(k_zero_bytes, grid, blk, 0, c.st, P->d_det, c.n);  // clip flags of the preconditioned method
  hipLaunchKernelGGL(k_pk_seed, grid, blk, 0, c.st, (const double*)p, P->d_part, c.n);
  if (force) {
    hipLaunchKernelGGL(k_pk_scale0, grid, blk, 0, c.st, p, P->d_state, P->d_part, c.nb, c.n);
    // the first gap folds sum p from here: that of the scaled p
    hipLaunchKernelGGL(k_pk_seed, grid, blk, 0, c.st, (const double*)p, P->d_part, c.n);
  }
  hipLaunchKernelGGL(k_mask_from_p, grid, blk, 0, c.st, (const double*)p, P->d_mask2, c.n);
  CB_HIP(apply64(c, p, (double*)P->d_u, nullptr));
  SolverState s;
  // Automatic.  From a start far from the contact set (the uniform force
  // start, the overlap of displacement control), two-phase: while the set
  // changes, each change restarts the directions, and the cheap plain (or,
  // on stiff thin coatings, layer-preconditioned) iteration wins; once the
  // set holds, the inverse symbol finishes the solve fastest.  From a
  // start whose support is close to the contact (a caller's guess, the
  // estimated force start), the inverse symbol throughout (N = 1024 force
  // set, the 26 other coatings: 281 iterations against 309 two-phase),
  // except on stiff thin coatings, where two-phase is kept (434 against
  // 810 over the set's 6).
  const int two = 3 + P->precond_auto;
  const int pk = op.precond == 3 ? two
                 : op.precond >= 0 ? op.precond
                 : (near && P->precond_auto == 0) ? 2 : two;
  auto enq = [&](int n) { return pk_enqueue_chunk<TD>(c, p, f, force, pk, n); };
  auto enq1 = [&](int n) { return pk_enqueue_chunk<TD>(c, p, f, force, pk, n, true); };
  // kinds: 0..19 (force + 4 mode), and 32 + that for the second phase
  const int kind = (force ? 1 : 0) + 4 * pk;
  if (int rc = run_chunks(P, kind, 32 + kind, p, f, nullptr, op.chunk, op.max_iter, enq, enq1, &s, 1.0)) return rc;
  const int status = s.nonfinite ? CB_E_NONFINITE : (s.done ? CB_OK : CB_E_NOCONV);
  hipLaunchKernelGGL(k_pk_pending_scale, grid, blk, 0, c.st, p, (double*)P->d_u, P->d_state, c.n);
  hipLaunchKernelGGL(k_stats, grid, blk, 0, c.st, (const double*)p, (const double*)P->d_u,
                     (const unsigned char*)nullptr, P->d_part, c.n);
  hipLaunchKernelGGL(k_fold_misc<4>, dim3(1), blk, 0, c.st, P->d_part, c.nb, 8);
  double s4[4];
  if (int rc = read_scratch(c, s4, 4)) return rc;
  if (mask) hipLaunchKernelGGL(k_mask_from_p, grid, blk, 0, c.st, (const double*)p, mask, c.n);
  CB_HIP(hipStreamSynchronize(c.st));
  res->status = status;
  res->iters = s.iters;
  res->rounds = 0;
  res->resid = s.resid;
  res->F = dA * s4[0];
  res->d = force ? s.d : target;
  res->area = dA * s4[1];
  res->U_el = 0.5 * dA * s4[2];
  res->U_ad = 0.0;
  res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (status != CB_OK)
    return cb_fail(status, status == CB_E_NOCONV ? "iteration limit reached" : "non-finite value in iteration");
  return CB_OK;
}

// CG on the fixed set S; x in/out.  The recurrence residual is confirmed by
// the true residual b - K x computed with an FP64 convolution; if that is
// still above tol the CG restarts from x (iterative refinement, at most
// SET_REFINE restarts).  A true residual still above tol after the last
// restart is CB_E_NOCONV.
constexpr int SET_REFINE = 4;
template <typename TD>
// `pending` (nullable): host copy of the previous round's detach/attach
// counts, read with this call's first state read; if both are zero that
// round changed nothing and the call stops there (*unchanged = true) with
// u = K x of the unchanged state.  On CB_OK, u = K x (the final check).
static int set_solve(const Ctx& c, const double* f, double d, const unsigned char* S, double* x, double tol,
                     int max_iter, int chunk, int pk, int& iters, double& resid, const double* pending = nullptr,
                     bool* unchanged = nullptr) {
  cb_plan_s* P = c.P;
  double* u = (double*)P->d_u;
  double* r = (double*)P->d_g;
  TD* z = (TD*)P->d_t;
  const dim3 grid(c.nb), blk(RT);
  int budget = max_iter;
  for (int attempt = 0; attempt <= SET_REFINE; attempt++) {
    if (int rc = write_state(P, base_state(P, tol, d, false, 0.0))) return rc;
    hipLaunchKernelGGL(k_zero_off, grid, blk, 0, c.st, x, S, c.n);
    CB_HIP(apply64(c, x, u, nullptr));
    hipLaunchKernelGGL(k_mcg_init<TD>, grid, blk, 0, c.st, f, (const double*)u, S, r, z, P->d_state, P->d_part, c.n);
    hipLaunchKernelGGL(k_mcg_init_fin, dim3(1), blk, 0, c.st, P->d_state, P->d_part, c.nb);
    SolverState s;
    if (int rc = read_state(P, &s)) return rc;
    if (attempt == 0 && pending && pending[0] == 0.0 && pending[1] == 0.0) {
      *unchanged = true;
      return CB_OK;
    }
    if (s.nonfinite) return CB_E_NONFINITE;
    resid = s.resid;
    // converged on the true residual; or out of refinement restarts or
    // iterations with the true residual still above tol
    if (s.done) return CB_OK;
    if (attempt == SET_REFINE || budget <= 0) return CB_E_NOCONV;
    if (pk > 0) {  // y = M^-1 r (z holds r in the direction type), z = y on S
      CB_HIP(apply_pc(c, z, P->d_y, nullptr, pk == 2 ? P->d_pinv : P->d_ptable));
      hipLaunchKernelGGL(k_mcg_pc0<TD>, grid, blk, 0, c.st, (const double*)r, (const TD*)P->d_y, z, S, P->d_state,
                         P->d_part, c.n);
    }
    auto enq = [&](int n) { return mcg_enqueue_chunk<TD>(c, x, S, n, pk); };
    if (int rc = run_chunks(P, 2 + 16 * pk, 2 + 16 * pk, x, S, f, chunk, budget, enq, enq, &s, resid)) return rc;
    iters += s.iters;
    budget -= s.iters;
    if (s.nonfinite) return CB_E_NONFINITE;
    if (!s.done) return CB_E_NOCONV;
  }
  return CB_OK;
}

// One adhesive displacement step on the state (S, p); S/Salt are the two
// contact-set buffers (swapped as rounds proceed).
template <typename TD>
static int adhesive_step(const Ctx& c, const double* f, double d, double* p, unsigned char*& S,
                         unsigned char*& Salt, bool attach_start, const Opts& op, cb_result* res) {
  cb_plan_s* P = c.P;
  double* u = (double*)P->d_u;
  const double dA = P->dx * P->dx;
  const dim3 grid(c.nb), blk(RT);
  int iters = 0, rounds = 0, status = CB_OK;
  double resid = 0.0;
  if (attach_start) {
    CB_HIP(apply64(c, p, u, nullptr));
    hipLaunchKernelGGL(k_attach_start, grid, blk, 0, c.st, f, (const double*)u, d, S, P->d_det, p, c.n);
  }
  // Each round: the fixed-set solve (its final check leaves u = K p), then
  // the Eq. 12 detachment and attachment.  The round's counts are not read
  // on their own: they travel with the next solve's first state read, and a
  // round that changed nothing ends the step there (that solve's start
  // only recomputes u of the unchanged state).
  double* pending = reinterpret_cast<double*>(&P->h_state[1]);
  bool have_pending = false;
  while (true) {
    // fixed-set CG: automatic = preconditioned by the inverse symbol (on a
    // fixed set it needs 3-7x fewer iterations than plain CG)
    const int pk = op.precond >= 0 ? op.precond : 2;
    bool unchanged = false;
    const int rc = set_solve<TD>(c, f, d, S, p, op.tol, op.max_iter, op.chunk, pk, iters, resid,
                                 have_pending ? pending : nullptr, &unchanged);
    if (rc != CB_OK) { status = rc; break; }
    if (unchanged) break;
    rounds++;
    hipLaunchKernelGGL(k_detach_attach, grid, blk, 0, c.st, f, (const double*)u, p, (const unsigned char*)S, Salt,
                       P->d_det, P->N, d, P->sigma_c, op.atol, P->d_part);
    hipLaunchKernelGGL(k_fold_misc<2>, dim3(1), blk, 0, c.st, P->d_part, c.nb, 0);
    std::swap(S, Salt);
    if (rounds == op.max_rounds) {
      double ch[2];
      if (int e = read_scratch(c, ch, 2)) return e;
      if (ch[0] != 0.0 || ch[1] != 0.0) status = CB_E_NOCONV;
      break;
    }
    CB_HIP(hipMemcpyAsync(pending, P->d_part + SCRATCH_OFF, 2 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    have_pending = true;
  }
  hipLaunchKernelGGL(k_stats, grid, blk, 0, c.st, (const double*)p, (const double*)u, (const unsigned char*)S,
                     P->d_part, c.n);
  hipLaunchKernelGGL(k_fold_misc<4>, dim3(1), blk, 0, c.st, P->d_part, c.nb, 8);
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

template <typename TD>
static int adhesive_indent(cb_plan_s* P, const double* f, double d, double* p, unsigned char* mask_io,
                           const cb_solve_opts* o, cb_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c = make_ctx(P);
  const Opts op = fill_opts(P, o);
  *res = cb_result{};
  if (op.precond < -1 || op.precond > 2) return cb_fail(CB_E_INVALID, "precond must be -1, 0, 1 or 2");
  if (int rc = enter(P)) return rc;
  unsigned char* S = P->d_mask;
  unsigned char* Salt = P->d_mask2;
  hipLaunchKernelGGL(k_mask_overlap, dim3(c.nb), dim3(RT), 0, c.st, f, d, S, P->d_det, p, c.n);
  const int rc = adhesive_step<TD>(c, f, d, p, S, Salt, false, op, res);
  if (mask_io) CB_HIP(hipMemcpyAsync(mask_io, S, c.n, hipMemcpyDeviceToDevice, c.st));
  CB_HIP(hipStreamSynchronize(c.st));
  res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rc != CB_OK) return cb_fail(rc, "adhesive solve did not converge");
  return CB_OK;
}

// Adhesive force control (stable branch, F > 0).  The single adhesive
// solve at approach d (the geometric overlap, then the Eq. 12 detach
// rounds) defines F(d), which grows with d on the stable branch.  Adhesion
// lowers the force at a given approach, so the non-adhesive approach for F
// starts the bracket from below; the upper end is found by doubling steps,
// then Illinois regula falsi narrows it.  F(d) steps where a cell attaches
// or detaches, so the search stops when |F(d) - F| <= 1e-6 F or when the
// bracket has shrunk to 1e-13 of its first width; the result is the single
// solve at the d whose force came closest.
template <typename TD>
static int adhesive_force(cb_plan_s* P, const double* f, double F, double* p, unsigned char* mask_io,
                          const cb_solve_opts* o, cb_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  int iters = 0, rounds = 0;
  cb_result r{};
  if (int rc = pk_solve<TD>(P, f, F, true, p, nullptr, o, &r)) return rc;
  iters += r.iters;
  // the profile's lowest point: the non-adhesive penetration r.d - fmin
  // sets the scale of the bracket search
  Ctx c = make_ctx(P);
  hipLaunchKernelGGL(k_minmax, dim3(c.nb), dim3(RT), 0, c.st, f, nullptr, P->d_part, c.n);
  hipLaunchKernelGGL(k_fold_misc<4>, dim3(1), dim3(RT), 0, c.st, P->d_part, c.nb, 15);
  double mm[4];
  if (int rc = read_scratch(c, mm, 4)) return rc;
  const double fmin = -mm[0];
  double best_d = 0.0, best_err = INFINITY;
  auto eval = [&](double d, double* Fd) -> int {
    cb_result q{};
    const int rc = adhesive_indent<TD>(P, f, d, p, mask_io, o, &q);
    iters += q.iters;
    rounds += q.rounds;
    if (rc != CB_OK) return rc;
    *Fd = q.F;
    *res = q;
    if (std::fabs(q.F - F) < best_err) {
      best_err = std::fabs(q.F - F);
      best_d = d;
    }
    return CB_OK;
  };
  const double scale = std::max(0.05 * (r.d - fmin), 1e-9 * P->L);
  double dlo = r.d, Flo = 0.0, step = scale;
  if (int rc = eval(dlo, &Flo)) return rc;
  for (int k = 0; Flo >= F; k++) {  // rarely: the adhesive force already exceeds F
    if (k == 60) return cb_fail(CB_E_NOCONV, "adhesive force control: no lower bracket");
    dlo -= step;
    step *= 2.0;
    if (int rc = eval(dlo, &Flo)) return rc;
  }
  step = scale;
  double dhi = dlo + step, Fhi = 0.0;
  if (int rc = eval(dhi, &Fhi)) return rc;
  for (int k = 0; Fhi < F; k++) {
    if (k == 60) return cb_fail(CB_E_NOCONV, "adhesive force control: no upper bracket");
    dlo = dhi;
    Flo = Fhi;
    step *= 2.0;
    dhi = dlo + step;
    if (int rc = eval(dhi, &Fhi)) return rc;
  }
  const double width0 = dhi - dlo;
  int side = 0;
  double last_d = dhi;
  for (int k = 0; k < 200 && best_err > 1e-6 * F && dhi - dlo > 1e-13 * width0; k++) {
    double d = dhi - (Fhi - F) * (dhi - dlo) / (Fhi - Flo);
    if (!(d > dlo && d < dhi)) d = 0.5 * (dlo + dhi);
    double Fd = 0.0;
    if (int rc = eval(d, &Fd)) return rc;
    last_d = d;
    if (Fd < F) {
      if (side == -1) Fhi = F + 0.5 * (Fhi - F);
      dlo = d;
      Flo = Fd;
      side = -1;
    } else {
      if (side == 1) Flo = F + 0.5 * (Flo - F);
      dhi = d;
      Fhi = Fd;
      side = 1;
    }
  }
  if (best_d != last_d) {
    double Fd = 0.0;
    if (int rc = eval(best_d, &Fd)) return rc;
  }
  res->iters = iters;
  res->rounds = rounds;
  res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return CB_OK;
}

// Adhesive force control with F <= 0: the pull-off under force control
// (Sec. 3.1, Eq. 19).  Preload by the single adhesive solve at d_pre, then
// the quasi-static displacement steps of the paper's retraction, each
// carrying the state; in the first step at or below F, regula falsi over
// single steps from the state of the step before.  Contact lost first:
// F lies below the pull-off force, the step of the lowest force is
// returned with CB_E_NOCONV.
template <typename TD>
static int adhesive_retract(cb_plan_s* P, const double* f, double F, double* p, unsigned char* mask_io,
                            const cb_solve_opts* o, cb_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c = make_ctx(P);
  Opts op = fill_opts(P, o);
  *res = cb_result{};
  if (op.precond < -1 || op.precond > 2) return cb_fail(CB_E_INVALID, "precond must be -1, 0, 1 or 2");
  if (!P->d_save_p[0]) return cb_fail(CB_E_STATE, "adhesive plan without retraction buffers");
  if (int rc = enter(P)) return rc;
  hipLaunchKernelGGL(k_minmax, dim3(c.nb), dim3(RT), 0, c.st, f, nullptr, P->d_part, c.n);
  hipLaunchKernelGGL(k_fold_misc<4>, dim3(1), dim3(RT), 0, c.st, P->d_part, c.nb, 15);
  double mm[4];
  if (int rc = read_scratch(c, mm, 4)) return rc;
  if (mm[2] > 0.0) return cb_fail(CB_E_NONFINITE, "profile f contains NaN/Inf");
  const double fmin = -mm[0];
  int iters = 0, rounds = 0;
  double d_pre = op.preload_d;
  if (!(d_pre > fmin)) {
    // the approach at which the non-adhesive solve carries the preload force
    cb_solve_opts o2{};
    if (o) o2 = *o;
    o2.init = 0;
    cb_result r{};
    const double Fpre = std::max(4.0 * std::fabs(F), M_PI * P->dgamma * P->L / 2.0);
    if (int rc = pk_solve<TD>(P, f, Fpre, true, p, nullptr, &o2, &r)) return rc;
    iters += r.iters;
    d_pre = r.d;
  }
  const size_t n8 = (size_t)c.n * 8;
  double* sp[2] = {P->d_save_p[0], P->d_save_p[1]};   // 0: step before, 1: best
  unsigned char* sS[2] = {P->d_save_S[0], P->d_save_S[1]};
  unsigned char* S = P->d_mask;
  unsigned char* Salt = P->d_mask2;
  auto save = [&](int q) -> int {
    CB_HIP(hipMemcpyAsync(sp[q], p, n8, hipMemcpyDeviceToDevice, c.st));
    CB_HIP(hipMemcpyAsync(sS[q], S, c.n, hipMemcpyDeviceToDevice, c.st));
    return CB_OK;
  };
  auto restore = [&](int q) -> int {
    CB_HIP(hipMemcpyAsync(p, sp[q], n8, hipMemcpyDeviceToDevice, c.st));
    CB_HIP(hipMemcpyAsync(S, sS[q], c.n, hipMemcpyDeviceToDevice, c.st));
    return CB_OK;
  };
  auto step = [&](double d, bool from_overlap, cb_result* q) -> int {
    if (from_overlap)
      hipLaunchKernelGGL(k_mask_overlap, dim3(c.nb), dim3(RT), 0, c.st, f, d, S, P->d_det, p, c.n);
    const int rc = adhesive_step<TD>(c, f, d, p, S, Salt, !from_overlap, op, q);
    iters += q->iters;
    rounds += q->rounds;
    return rc;
  };
  cb_result q{}, best{};
  if (int rc = step(d_pre, true, &q)) return cb_fail(rc, "adhesive preload did not converge");
  best = q;
  if (int rc = save(0)) return rc;
  if (int rc = save(1)) return rc;
  const double dd = (d_pre - fmin) / 32.0;
  // force tolerance of the refinement: 1e-6 of |F|, or of 1e-3 of the
  // preload force when F is near zero
  const double ftol = 1e-6 * std::max(std::fabs(F), 1e-3 * std::fabs(q.F));
  double d = d_pre, Fc = q.F;
  int status = CB_E_NOCONV;
  bool found = false;
  for (int k = 0; k < 4096 && !found; k++) {
    const double dn = d - dd;
    if (int rc = step(dn, false, &q)) return cb_fail(rc, "adhesive retraction step did not converge");
    if (q.F < best.F) {
      best = q;
      if (int rc = save(1)) return rc;
    }
    if (q.F <= F) {
      // refine inside (dn, d) from the state of the step before; the best
      // match so far is kept in slot 1
      double lo = dn, hi = d, Flo = q.F, Fhi = Fc;
      cb_result match = q;
      if (int rc = save(1)) return rc;
      int side = 0;
      for (int it = 0; it < 200; it++) {
        if (std::fabs(match.F - F) <= ftol || hi - lo <= 1e-13 * dd) break;
        double x = hi - (Fhi - F) * (hi - lo) / (Fhi - Flo);
        if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
        if (int rc = restore(0)) return rc;
        if (int rc = step(x, false, &q)) return cb_fail(rc, "adhesive retraction step did not converge");
        if (std::fabs(q.F - F) < std::fabs(match.F - F)) {
          match = q;
          if (int rc = save(1)) return rc;
        }
        if (q.F < F) {
          if (side == -1) Fhi = F + 0.5 * (Fhi - F);
          lo = x;
          Flo = q.F;
          side = -1;
        } else {
          if (side == 1) Flo = F + 0.5 * (Flo - F);
          hi = x;
          Fhi = q.F;
          side = 1;
        }
      }
      best = match;
      status = CB_OK;
      found = true;
      break;
    }
    if (!(q.area > 0.0)) break;  // contact lost: F is below the pull-off force
    if (int rc = save(0)) return rc;
    d = dn;
    Fc = q.F;
  }
  if (int rc = restore(1)) return rc;
  if (mask_io) CB_HIP(hipMemcpyAsync(mask_io, S, c.n, hipMemcpyDeviceToDevice, c.st));
  CB_HIP(hipStreamSynchronize(c.st));
  *res = best;
  res->status = status;
  res->iters = iters;
  res->rounds = rounds;
  res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (status != CB_OK)
    return cb_fail(status, "pull-off before the force was reached: the lowest force of the retraction is above F");
  return CB_OK;
}

template <typename TD>
static int sweep_impl(cb_plan_s* P, const double* f, const double* dsteps, int nsteps, double* p,
                      unsigned char* mask, const cb_solve_opts* o, cb_result* out) {
  Ctx c = make_ctx(P);
  const Opts op = fill_opts(P, o);
  if (op.precond < -1 || op.precond > 2) return cb_fail(CB_E_INVALID, "precond must be -1, 0, 1 or 2");
  if (int rc = enter(P)) return rc;
  unsigned char* S = mask;
  unsigned char* Salt = P->d_mask;
  int first_err = CB_OK;
  for (int k = 0; k < nsteps; k++) {
    const auto t0 = std::chrono::steady_clock::now();
    out[k] = cb_result{};
    const int rc = adhesive_step<TD>(c, f, dsteps[k], p, S, Salt, true, op, &out[k]);
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

extern "C" int cb_solve_indent(cb_plan P, const double* f, double d, double* p_io, unsigned char* mask_io,
                               const cb_solve_opts* o, cb_result* res) {
  if (!P || !f || !p_io || !res) return cb_fail(CB_E_INVALID, "null argument");
  if (!aligned16(f) || !aligned16(p_io) || (mask_io && !aligned16(mask_io)))
    return cb_fail(CB_E_INVALID, "f, p and mask must be 16-byte aligned");
  if (!std::isfinite(d)) return cb_fail(CB_E_INVALID, "d must be finite");
  if (P->dgamma > 0.0) {
    if (P->precision == CB_FP64) return adhesive_indent<double>(P, f, d, p_io, mask_io, o, res);
    return adhesive_indent<float>(P, f, d, p_io, mask_io, o, res);
  }
  if (P->precision == CB_FP64) return pk_solve<double>(P, f, d, false, p_io, mask_io, o, res);
  return pk_solve<float>(P, f, d, false, p_io, mask_io, o, res);
}

extern "C" int cb_solve_force(cb_plan P, const double* f, double F, double* p_io, unsigned char* mask_io,
                              const cb_solve_opts* o, cb_result* res) {
  if (!P || !f || !p_io || !res) return cb_fail(CB_E_INVALID, "null argument");
  if (!aligned16(f) || !aligned16(p_io) || (mask_io && !aligned16(mask_io)))
    return cb_fail(CB_E_INVALID, "f, p and mask must be 16-byte aligned");
  if (!std::isfinite(F)) return cb_fail(CB_E_INVALID, "F must be finite");
  if (P->dgamma > 0.0) {
    if (F <= 0.0) {
      if (P->precision == CB_FP64) return adhesive_retract<double>(P, f, F, p_io, mask_io, o, res);
      return adhesive_retract<float>(P, f, F, p_io, mask_io, o, res);
    }
    if (P->precision == CB_FP64) return adhesive_force<double>(P, f, F, p_io, mask_io, o, res);
    return adhesive_force<float>(P, f, F, p_io, mask_io, o, res);
  }
  if (F < 0.0) return cb_fail(CB_E_INVALID, "F must be >= 0 on a non-adhesive plan");
  if (P->precision == CB_FP64) return pk_solve<double>(P, f, F, true, p_io, mask_io, o, res);
  return pk_solve<float>(P, f, F, true, p_io, mask_io, o, res);
}

extern "C" int cb_sweep(cb_plan P, const double* f, const double* d_steps, int nsteps, double* p_state,
                        unsigned char* mask_state, const cb_solve_opts* o, cb_result* per_step) {
  if (!P || !f || !d_steps || !p_state || !mask_state || !per_step || nsteps < 0)
    return cb_fail(CB_E_INVALID, "null argument or negative step count");
  if (!aligned16(f) || !aligned16(p_state) || !aligned16(mask_state))
    return cb_fail(CB_E_INVALID, "f, p and mask must be 16-byte aligned");
  if (!(P->dgamma > 0.0)) return cb_fail(CB_E_UNSUPPORTED, "sweep needs an adhesive plan (dgamma > 0)");
  for (int k = 0; k < nsteps; k++)
    if (!std::isfinite(d_steps[k])) return cb_fail(CB_E_INVALID, "non-finite displacement step");
  if (P->precision == CB_FP64) return sweep_impl<double>(P, f, d_steps, nsteps, p_state, mask_state, o, per_step);
  return sweep_impl<float>(P, f, d_steps, nsteps, p_state, mask_state, o, per_step);
}
