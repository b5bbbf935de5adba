// Learned warm start for the contact solve: a small U-Net (16 channels,
// twelve 3x3 convolutions, 256 -> 32 -> 256) mapping the gap field and the
// problem scalars to an initial pressure field.  Forward, backward and Adam
// run in these kernels; activations are BF16 (NHWC, 16 channels), every
// convolution is an implicit GEMM on the BF16 matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation), gradients and master
// weights are FP32.  The network definition is the one of the FP64
// reference used by the tests (16 channels everywhere, skip added before
// the decoder ReLU, softplus head normalised to unit mean).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace cbnet {

constexpr int C = 16;
constexpr int NLAYER = 12;
constexpr int LW = 9 * C * C;        // weights per layer
constexpr int LP = LW + C;           // parameters per layer
constexpr int NPARAM = NLAYER * LP;
constexpr int WAVES = 4;             // waves per block in the conv kernels
constexpr int WG_PIX = 4096;         // pixels per wave in the weight-gradient kernel

typedef unsigned short u16;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u16 f2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((unsigned)b << 16); }

// pixel q of the flattened (n, H, W) grid shifted by tap; -1 if outside
__device__ __forceinline__ int shifted(int q, int tap, int H, int W) {
  const int HW = H * W;
  const int img = q / HW, r = q - img * HW;
  const int y = r / W, x = r - y * W;
  const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
  if (yy < 0 || yy >= H || xx < 0 || xx >= W) return -1;
  return img * HW + yy * W + xx;
}

// y[q, co] = bias[co] + sum_tap sum_ci Wt[tap][co][ci] x[q + off(tap), ci]
// (+ skip[q, co]) (relu); one wave per 16-pixel tile.  MFMA operand layout
// (16x16x16 bf16): lane l holds A[i = l%16][k = 4(l/16)+j], B[k = 4(l/16)+j]
// [n = l%16] and D[i = 4(l/16)+j][n = l%16], j = 0..3.
template <bool RELU>
__global__ void __launch_bounds__(64 * WAVES)
k_conv(const u16* __restrict__ X, const u16* __restrict__ Wt, const float* __restrict__ bias,
       const u16* __restrict__ skip, u16* __restrict__ Yb, float* __restrict__ Yf, int P, int H, int W) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * WAVES + (threadIdx.x >> 6);
  if (tile * 16 >= P) return;
  const int i = lane & 15, kg = lane >> 4;
  s4 b[9];
#pragma unroll
  for (int tap = 0; tap < 9; tap++)
    b[tap] = *reinterpret_cast<const s4*>(Wt + (tap * C + i) * C + 4 * kg);
  // the epilogue's operands (bias, skip) are loaded with the others
  const int co = i;
  const float bb = bias ? bias[co] : 0.f;
  // (unconditional: without a skip the input, of the same shape, is read
  // and its value dropped, so that no branch ends in a wait)
  const u16* sks = skip ? skip : X;
  float sk[4];
#pragma unroll
  for (int j = 0; j < 4; j++) sk[j] = bf2f(sks[(size_t)(tile * 16 + 4 * kg + j) * C + co]);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  const int q = tile * 16 + i;
  // the nine taps' loads are unconditional (a tap outside the image reads
  // the pixel itself and is zeroed after the load), so that they go out
  // together instead of one round trip per tap behind a branch
  s4 a[9];
#pragma unroll
  for (int tap = 0; tap < 9; tap++) {
    const int qs = shifted(q, tap, H, W);
    a[tap] = *reinterpret_cast<const s4*>(X + (size_t)(qs >= 0 ? qs : q) * C + 4 * kg);
    if (qs < 0) a[tap] = s4{0, 0, 0, 0};
  }
#pragma unroll
  for (int tap = 0; tap < 9; tap++) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[tap], b[tap], acc, 0, 0, 0);
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int qo = tile * 16 + 4 * kg + j;
    float v = acc[j] + bb;
    if (skip) v += sk[j];
    if (RELU) v = v > 0.f ? v : 0.f;
    if (Yb) Yb[(size_t)qo * C + co] = f2bf(v);
    if (Yf) Yf[(size_t)qo * C + co] = v;
  }
}

// Weight gradient: part[w][tap][co][ci] = sum over the wave's pixels of
// dA[q, co] x[q + off(tap), ci]; partb[w][co] = sum dA[q, co].  MFMA with
// M = co, N = ci, K = 16 pixels per step.
__global__ void __launch_bounds__(64 * WAVES)
k_conv_wgrad(const u16* __restrict__ dA, const u16* __restrict__ X, float* __restrict__ part,
             float* __restrict__ partb, int P, int H, int W, int nw) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * WAVES + (threadIdx.x >> 6);
  if (w >= nw) return;
  const int i = lane & 15, kg = lane >> 4;
  f4 acc[9];
#pragma unroll
  for (int tap = 0; tap < 9; tap++) acc[tap] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const int q0 = w * WG_PIX;
  const int q1 = min(q0 + WG_PIX, P);
  for (int qb = q0; qb < q1; qb += 16) {
    s4 a;
    short av[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int q = qb + 4 * kg + j;
      av[j] = (short)dA[(size_t)q * C + i];  // A[co = i][k = pixel]
      bsum += bf2f((u16)av[j]);
    }
    a = s4{av[0], av[1], av[2], av[3]};
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
      short bv[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int qs = shifted(qb + 4 * kg + j, tap, H, W);
        bv[j] = qs >= 0 ? (short)X[(size_t)qs * C + i] : (short)0;  // B[k = pixel][ci = i]
      }
      acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, s4{bv[0], bv[1], bv[2], bv[3]}, acc[tap], 0, 0, 0);
    }
  }
  // D[co = 4 kg + j][ci = i]
#pragma unroll
  for (int tap = 0; tap < 9; tap++)
#pragma unroll
    for (int j = 0; j < 4; j++) part[((size_t)w * 9 + tap) * C * C + (4 * kg + j) * C + i] = acc[tap][j];
  // bias: lanes with the same i = co hold disjoint pixel groups kg
  bsum += __shfl_xor(bsum, 16, 64);
  bsum += __shfl_xor(bsum, 32, 64);
  if (kg == 0) partb[(size_t)w * C + i] = bsum;
}

// grad[layer] = sum over waves (fixed order) of the partials
__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ partb, int nw,
                               float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < LW) {
    float s = 0.f;
    for (int w = 0; w < nw; w++) s += part[(size_t)w * LW + e];
    grad[e] = s;
  } else if (e < LP) {
    const int c = e - LW;
    float s = 0.f;
    for (int w = 0; w < nw; w++) s += partb[(size_t)w * C + c];
    grad[e] = s;
  }
}

// dA = bf16(dY * (Y > 0)); dskip += dY * (Y > 0) when given
__global__ void k_relu_bwd(const float* __restrict__ dY, const u16* __restrict__ Y, u16* __restrict__ dA,
                           float* __restrict__ dskip, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const float v = bf2f(Y[e]) > 0.f ? dY[e] : 0.f;
    dA[e] = f2bf(v);
    if (dskip) dskip[e] += v;
  }
}
__global__ void k_to_bf16(const float* __restrict__ x, u16* __restrict__ y, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    y[e] = f2bf(x[e]);
}
__global__ void k_zero(float* __restrict__ x, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    x[e] = 0.f;
}
// 2x2 average pool (n, H, W) -> (n, H/2, W/2), 16 channels
__global__ void k_pool(const u16* __restrict__ X, u16* __restrict__ Y, int n, int H, int W) {
  const int Ho = H / 2, Wo = W / 2;
  const long long tot = (long long)n * Ho * Wo * C;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int c = e % C;
    long long r = e / C;
    const int x = r % Wo;
    r /= Wo;
    const int y = r % Ho;
    const int img = r / Ho;
    const size_t b = (((size_t)img * H + 2 * y) * W + 2 * x) * C + c;
    const float s = bf2f(X[b]) + bf2f(X[b + C]) + bf2f(X[b + (size_t)W * C]) + bf2f(X[b + (size_t)W * C + C]);
    Y[e] = f2bf(0.25f * s);
  }
}
// dX (fine) += dY (coarse) / 4
__global__ void k_pool_bwd(const float* __restrict__ dY, float* __restrict__ dX, int n, int H, int W) {
  const long long tot = (long long)n * H * W * C;
  const int Wo = W / 2, Ho = H / 2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int c = e % C;
    long long r = e / C;
    const int x = r % W;
    r /= W;
    const int y = r % H;
    const int img = r / H;
    dX[e] += 0.25f * dY[(((size_t)img * Ho + y / 2) * Wo + x / 2) * C + c];
  }
}
// nearest 2x upsample (n, H, W) -> (n, 2H, 2W)
__global__ void k_up(const u16* __restrict__ X, u16* __restrict__ Y, int n, int H, int W) {
  const int Ho = 2 * H, Wo = 2 * W;
  const long long tot = (long long)n * Ho * Wo * C;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int c = e % C;
    long long r = e / C;
    const int x = r % Wo;
    r /= Wo;
    const int y = r % Ho;
    const int img = r / Ho;
    Y[e] = X[(((size_t)img * H + y / 2) * W + x / 2) * C + c];
  }
}
// dX (coarse) = sum of the 2x2 fine gradients
__global__ void k_up_bwd(const float* __restrict__ dY, float* __restrict__ dX, int n, int H, int W) {
  const long long tot = (long long)n * H * W * C;
  const int Wf = 2 * W;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int c = e % C;
    long long r = e / C;
    const int x = r % W;
    r /= W;
    const int y = r % H;
    const int img = r / H;
    const size_t b = (((size_t)img * 2 * H + 2 * y) * Wf + 2 * x) * C + c;
    dX[e] = dY[b] + dY[b + C] + dY[b + (size_t)Wf * C] + dY[b + (size_t)Wf * C + C];
  }
}

__device__ __forceinline__ float softplusf(float z) { return z > 20.f ? z : log1pf(expf(z)); }

// Head: per sample (one block), q = softplus(z), p^ = q / mean q, the
// target normalised to unit mean t^ = t / mean t, loss_n = sum (p^ - t^)^2
// / sum t^^2; dz (for the batch mean of loss_n) goes into channel 0 of dY,
// the other channels are zero.  Fixed-order FP64 block reductions.
__device__ __forceinline__ void block_sum3(double (*sh)[256], double& a, double& b, double& c) {
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < 3; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    }
    __syncthreads();
  }
  a = sh[0][0];
  b = sh[1][0];
  c = sh[2][0];
  __syncthreads();
}

__global__ void __launch_bounds__(256)
k_head_loss(const float* __restrict__ Z16, const float* __restrict__ t, float* __restrict__ dY, double* lossv,
            int HW, int n) {
  const int img = blockIdx.x;
  __shared__ double sh[3][256];
  const float* ti = t + (size_t)img * HW;
  double sq = 0.0, st = 0.0, stt = 0.0;
  for (int e = threadIdx.x; e < HW; e += 256) {
    sq += softplusf(Z16[((size_t)img * HW + e) * C]);
    const double tv = ti[e];
    st += tv;
    stt += tv * tv;
  }
  block_sum3(sh, sq, st, stt);
  const double m = sq / HW, ts = HW / st, tt = stt * ts * ts;
  double srr = 0.0, sdq = 0.0, unused = 0.0;
  for (int e = threadIdx.x; e < HW; e += 256) {
    const double q = softplusf(Z16[((size_t)img * HW + e) * C]);
    const double r = q / m - ti[e] * ts;
    srr += r * r;
    sdq += (2.0 * r / tt / n) * q;
  }
  block_sum3(sh, srr, sdq, unused);
  if (threadIdx.x == 0) lossv[img] = srr / tt;
  for (int e = threadIdx.x; e < HW; e += 256) {
    const size_t o = ((size_t)img * HW + e) * C;
    const float z = Z16[o];
    const double q = softplusf(z);
    const double r = q / m - ti[e] * ts;
    const double dph = 2.0 * r / tt / n;
    const double dq = dph / m - sdq / (m * m * HW);
    dY[o] = (float)(dq / (1.0 + exp(-(double)z)));
#pragma unroll
    for (int c = 1; c < C; c++) dY[o + c] = 0.f;
  }
}

// Adam on the flat FP32 parameters, then the BF16 forward copy [l][tap][co][ci]
// and the backward-data copy [l][8 - tap][ci][co].
__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NPARAM) return;
  const float gi = g[e];
  const float a = b1 * m1[e] + (1.f - b1) * gi;
  const float v = b2 * m2[e] + (1.f - b2) * gi * gi;
  m1[e] = a;
  m2[e] = v;
  prm[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}
__global__ void k_weights_bf16(const float* __restrict__ prm, u16* __restrict__ wf, u16* __restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NLAYER * LW) return;
  const int l = e / LW, r = e - l * LW;
  const int tap = r / (C * C), co = (r / C) % C, ci = r % C;
  const u16 v = f2bf(prm[l * LP + r]);
  wf[e] = v;
  wb[(size_t)l * LW + ((8 - tap) * C + ci) * C + co] = v;
}

// ---------------------------------------------------------------------------
// Warm-start input features and output prolongation
// ---------------------------------------------------------------------------
// Two-stage reductions for the warm start: RP blocks write one partial
// each; the consumer folds the RP partials in a fixed order.
constexpr int RP = 64;

struct Scalars {
  float s[8];
};

// The problems of one warm-start launch, by value: problem q of a launch is
// blockIdx.y; its slot in the net's buffers and partials is base + q.
constexpr int WS_MAX = 32;
struct WsProblem {
  const double* f;   // N x N profile
  double* p;         // N x N initial pressure (output)
  float* x;          // G x G x C features (output)
  int N;
  int guess;         // 0: the problem gets zeros (the solve takes its cold start)
  double L;
  Scalars sc;
};
struct WsBatch {
  WsProblem q[WS_MAX];
};

// partial minima of f over N*N (RP blocks per problem)
__global__ void __launch_bounds__(256) k_fmin(WsBatch B, int base, double* scratch) {
  __shared__ double sh[256];
  const WsProblem& P = B.q[blockIdx.y];
  double* part = scratch + (size_t)(base + blockIdx.y) * RP;
  // 16-byte loads, four independent minima per thread (n even: N x N, N >= 8)
  double m0 = INFINITY, m1 = INFINITY, m2 = INFINITY, m3 = INFINITY;
  const double2* f2 = reinterpret_cast<const double2*>(P.f);
  const int n2 = (P.N * P.N) >> 1, stride = RP * 256;
  int e = blockIdx.x * 256 + threadIdx.x;
  for (; e + stride < n2; e += 2 * stride) {
    const double2 a = f2[e], b = f2[e + stride];
    m0 = fmin(m0, a.x);
    m1 = fmin(m1, a.y);
    m2 = fmin(m2, b.x);
    m3 = fmin(m3, b.y);
  }
  if (e < n2) {
    const double2 a = f2[e];
    m0 = fmin(m0, a.x);
    m1 = fmin(m1, a.y);
  }
  const double m = fmin(fmin(m0, m1), fmin(m2, m3));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__device__ __forceinline__ double fold_min(const double* part) {
  double m = part[0];
  for (int b = 1; b < RP; b++) m = fmin(m, part[b]);
  return m;
}
__device__ __forceinline__ double fold_sum(const double* part) {
  double s = 0.0;
  for (int b = 0; b < RP; b++) s += part[b];
  return s;
}

// x[y][x][c] on the G x G net grid from the N x N profile: cell averages
// (N >= G) or nearest cells (N < G) of the gap g0 = f - min f, as three
// clipped channels g0/(s L) for s in {0.005, 0.02, 0.08}, then the
// problem scalars broadcast, remaining channels zero.
__global__ void k_features(WsBatch B, int base, int G, const double* scratch) {
  const WsProblem& P = B.q[blockIdx.y];
  const int N = P.N, tot = G * G;
  const double L = P.L;
  const double* __restrict__ f = P.f;
  __shared__ double f0_s;
  if (threadIdx.x == 0) f0_s = fold_min(scratch + (size_t)(base + blockIdx.y) * RP);
  __syncthreads();
  const double f0 = f0_s;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int y = e / G, xx = e % G;
    double g0;
    if (N >= G) {
      const int r = N / G;
      double s = 0.0;
      for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) s += f[(size_t)(y * r + a) * N + xx * r + b];
      g0 = s / (r * r) - f0;
    } else {
      const int r = G / N;
      g0 = f[(size_t)(y / r) * N + xx / r] - f0;
    }
    float* o = P.x + (size_t)e * C;
    o[0] = (float)fmin(g0 / (0.005 * L), 1.0);
    o[1] = (float)fmin(g0 / (0.02 * L), 1.0);
    o[2] = (float)fmin(g0 / (0.08 * L), 1.0);
#pragma unroll
    for (int c = 0; c < 8; c++) o[3 + c] = P.sc.s[c];
#pragma unroll
    for (int c = 11; c < C; c++) o[c] = 0.f;
  }
}

// partial sums of softplus(z) over the G x G head of each problem that
// gets a guess; softplus(z) itself is kept in sp (G x G, compact) for the
// prolongation
__global__ void __launch_bounds__(256) k_qmean(WsBatch B, int base, const float* __restrict__ head, int G,
                                               double* scratch_mean, float* __restrict__ sp_all) {
  if (!B.q[blockIdx.y].guess) return;
  const int i = base + blockIdx.y;
  const float* Z16 = head + (size_t)i * G * G * C;
  float* sp = sp_all + (size_t)i * G * G;
  double* part = scratch_mean + (size_t)i * RP;
  __shared__ double sh[256];
  double s = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < G * G; e += RP * 256) {
    const float q = softplusf(Z16[(size_t)e * C]);
    sp[e] = q;
    s += q;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// p[N x N] from the head output z (channel 0 of a G x G x 16 FP32 tensor):
// q = softplus(z) / mean(q), set to zero below cut, then bilinear
// (cell-centred) interpolation to N >= G, or cell averages for N < G.
// Unit mean before the cut; the solve rescales to the load.  A problem
// without a guess gets zeros.
// (sp = softplus(z), compact, from k_qmean: one evaluation per head pixel)
__device__ __forceinline__ double qcut(const float* sp, int G, int yy, int xx, double inv_mean, double cut) {
  yy = yy < 0 ? 0 : (yy >= G ? G - 1 : yy);
  xx = xx < 0 ? 0 : (xx >= G ? G - 1 : xx);
  const double q = sp[(size_t)yy * G + xx] * inv_mean;
  return q < cut ? 0.0 : q;
}
__global__ void k_prolong(WsBatch B, int base, const float* __restrict__ sp_all, int G,
                          const double* scratch_mean, double cut) {
  const WsProblem& P = B.q[blockIdx.y];
  const int N = P.N, tot = N * N;
  double* __restrict__ p = P.p;
  if (!P.guess) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) p[e] = 0.0;
    return;
  }
  const int i = base + blockIdx.y;
  const float* sp = sp_all + (size_t)i * G * G;
  __shared__ double im_s;
  if (threadIdx.x == 0) im_s = ((double)G * G) / fold_sum(scratch_mean + (size_t)i * RP);
  __syncthreads();
  const double im = im_s;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int y = e / N, x = e % N;
    double v;
    if (N >= G) {
      const double sy = (y + 0.5) * G / N - 0.5, sx = (x + 0.5) * G / N - 0.5;
      const int y0 = (int)floor(sy), x0 = (int)floor(sx);
      const double wy = sy - y0, wx = sx - x0;
      v = (1 - wy) * ((1 - wx) * qcut(sp, G, y0, x0, im, cut) + wx * qcut(sp, G, y0, x0 + 1, im, cut)) +
          wy * ((1 - wx) * qcut(sp, G, y0 + 1, x0, im, cut) + wx * qcut(sp, G, y0 + 1, x0 + 1, im, cut));
    } else {
      const int r = G / N;
      double s = 0.0;
      for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) s += qcut(sp, G, y * r + a, x * r + b, im, cut);
      v = s / (r * r);
    }
    p[e] = v;
  }
}

}  // namespace cbnet

using namespace cbnet;

struct cb_net_s {
  int batch = 0, H = 0, W = 0;
  hipStream_t stream = nullptr;
  float *prm = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  u16 *wf = nullptr, *wb = nullptr;
  int step = 0;
  // activations (bf16) per level l (H >> l): x0, h, s, p (pooled input), u, e
  u16 *x0 = nullptr;
  u16 *h[4] = {}, *s[4] = {}, *pin[4] = {}, *up[3] = {}, *e[3] = {};
  float* head = nullptr;          // batch x H x W x 16 fp32
  float *g0 = nullptr, *g1 = nullptr, *gs[4] = {};  // fp32 gradient buffers
  u16* ga = nullptr;              // bf16 relu-masked gradient
  float *wpart = nullptr, *bpart = nullptr;
  double* lossv = nullptr;
  double* lossh = nullptr;
  double* scratch = nullptr;
  float* feat = nullptr;
  float* sp = nullptr;            // batch x H x W fp32: softplus of the head's channel 0
  std::vector<void*> allocs;
};

static int net_alloc(cb_net_s* N, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) return cb_fail(CB_E_NOMEM, "net allocation failed");
  N->allocs.push_back(*p);
  return CB_OK;
}

static dim3 egrid(long long n) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

extern "C" int cb_net_num_params(void) { return NPARAM; }

extern "C" int cb_net_destroy(cb_net N) {
  if (!N) return CB_OK;
  (void)hipStreamSynchronize(N->stream);
  for (void* p : N->allocs) (void)hipFree(p);
  if (N->lossh) (void)hipHostFree(N->lossh);
  delete N;
  return CB_OK;
}

extern "C" int cb_net_create(cb_net* out, int batch, int H, int W, void* stream) {
  if (!out) return cb_fail(CB_E_INVALID, "null output");
  *out = nullptr;
  if (batch < 1 || H < 32 || W < 32 || (H % 32) || (W % 32) || H > 4096 || W > 4096)
    return cb_fail(CB_E_INVALID, "net grid: H and W multiples of 32 in [32, 4096]");
  auto* N = new (std::nothrow) cb_net_s();
  if (!N) return cb_fail(CB_E_NOMEM, "host allocation failed");
  N->batch = batch;
  N->H = H;
  N->W = W;
  N->stream = (hipStream_t)stream;
  const size_t px = (size_t)batch * H * W;
  int rc = CB_OK;
  auto A = [&](void** p, size_t bytes) {
    if (rc == CB_OK) rc = net_alloc(N, p, bytes);
  };
  A((void**)&N->prm, NPARAM * 4);
  A((void**)&N->grad, NPARAM * 4);
  A((void**)&N->m1, NPARAM * 4);
  A((void**)&N->m2, NPARAM * 4);
  A((void**)&N->wf, NLAYER * LW * 2);
  A((void**)&N->wb, NLAYER * LW * 2);
  A((void**)&N->x0, px * C * 2);
  for (int l = 0; l < 4; l++) {
    const size_t pl = px >> (2 * l);
    A((void**)&N->h[l], pl * C * 2);
    A((void**)&N->s[l], pl * C * 2);
    A((void**)&N->pin[l], pl * C * 2);
    A((void**)&N->gs[l], pl * C * 4);
  }
  for (int l = 0; l < 3; l++) {
    const size_t pl = px >> (2 * l);
    A((void**)&N->up[l], pl * C * 2);
    A((void**)&N->e[l], pl * C * 2);
  }
  A((void**)&N->head, px * C * 4);
  A((void**)&N->g0, px * C * 4);
  A((void**)&N->g1, px * C * 4);
  A((void**)&N->ga, px * C * 2);
  const size_t nw = (px + WG_PIX - 1) / WG_PIX + 1;
  A((void**)&N->wpart, nw * LW * 4);
  A((void**)&N->bpart, nw * C * 4);
  A((void**)&N->lossv, batch * 8);
  A((void**)&N->scratch, (size_t)2 * batch * RP * 8);
  A((void**)&N->feat, px * C * 4);
  A((void**)&N->sp, px * 4);
  if (rc == CB_OK && hipHostMalloc((void**)&N->lossh, batch * 8, 0) != hipSuccess) rc = cb_fail(CB_E_NOMEM, "pinned");
  if (rc == CB_OK && (hipMemset(N->m1, 0, NPARAM * 4) != hipSuccess || hipMemset(N->m2, 0, NPARAM * 4) != hipSuccess ||
                      hipMemset(N->prm, 0, NPARAM * 4) != hipSuccess))
    rc = cb_fail(CB_E_DEVICE, "memset failed");
  if (rc != CB_OK) {
    cb_net_destroy(N);
    return rc;
  }
  *out = N;
  return CB_OK;
}

extern "C" int cb_net_set_params(cb_net N, const float* params) {
  if (!N || !params) return cb_fail(CB_E_INVALID, "null argument");
  CB_HIP(hipMemcpyAsync(N->prm, params, NPARAM * 4, hipMemcpyDeviceToDevice, N->stream));
  hipLaunchKernelGGL(k_weights_bf16, dim3((NLAYER * LW + 255) / 256), dim3(256), 0, N->stream, N->prm, N->wf, N->wb);
  CB_HIP(hipMemsetAsync(N->m1, 0, NPARAM * 4, N->stream));
  CB_HIP(hipMemsetAsync(N->m2, 0, NPARAM * 4, N->stream));
  N->step = 0;
  CB_HIP(hipGetLastError());
  return CB_OK;
}

extern "C" int cb_net_get_params(cb_net N, float* params) {
  if (!N || !params) return cb_fail(CB_E_INVALID, "null argument");
  CB_HIP(hipMemcpyAsync(params, N->prm, NPARAM * 4, hipMemcpyDeviceToDevice, N->stream));
  return CB_OK;
}

static void conv(cb_net_s* N, int l, const u16* X, const u16* skip, bool relu, u16* Yb, float* Yf, int n, int H,
                 int W, bool bwd_data = false) {
  const int P = n * H * W;
  const int tiles = P / 16;
  const dim3 grid((tiles + WAVES - 1) / WAVES), blk(64 * WAVES);
  const u16* Wt = (bwd_data ? N->wb : N->wf) + (size_t)l * LW;
  const float* bias = bwd_data ? nullptr : N->prm + (size_t)l * LP + LW;
  if (relu) hipLaunchKernelGGL(k_conv<true>, grid, blk, 0, N->stream, X, Wt, bias, skip, Yb, Yf, P, H, W);
  else hipLaunchKernelGGL(k_conv<false>, grid, blk, 0, N->stream, X, Wt, bias, skip, Yb, Yf, P, H, W);
}

static void forward(cb_net_s* N, int n) {
  const int H = N->H, W = N->W;
  // encoder
  const u16* in = N->x0;
  for (int l = 0; l < 4; l++) {
    const int h = H >> l, w = W >> l;
    if (l > 0) {
      hipLaunchKernelGGL(k_pool, egrid((long long)n * h * w * C), dim3(256), 0, N->stream, N->s[l - 1], N->pin[l], n,
                         2 * h, 2 * w);
      in = N->pin[l];
    }
    conv(N, 2 * l, in, nullptr, true, N->h[l], nullptr, n, h, w);
    conv(N, 2 * l + 1, N->h[l], nullptr, true, N->s[l], nullptr, n, h, w);
  }
  // decoder: e[l] = relu(conv(up(prev)) + s[l]) for l = 2, 1, 0
  const u16* prev = N->s[3];
  for (int l = 2; l >= 0; l--) {
    const int h = H >> l, w = W >> l;
    hipLaunchKernelGGL(k_up, egrid((long long)n * h * w * C), dim3(256), 0, N->stream, prev, N->up[l], n, h / 2, w / 2);
    conv(N, 10 - l, N->up[l], N->s[l], true, N->e[l], nullptr, n, h, w);
    prev = N->e[l];
  }
  conv(N, 11, N->e[0], nullptr, false, nullptr, N->head, n, H, W);
}

static void wgrad(cb_net_s* N, int l, const u16* dA, const u16* X, int n, int H, int W) {
  const int P = n * H * W;
  const int nw = (P + WG_PIX - 1) / WG_PIX;
  hipLaunchKernelGGL(k_conv_wgrad, dim3((nw + WAVES - 1) / WAVES), dim3(64 * WAVES), 0, N->stream, dA, X, N->wpart,
                     N->bpart, P, H, W, nw);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((LP + 255) / 256), dim3(256), 0, N->stream, N->wpart, N->bpart, nw,
                     N->grad + (size_t)l * LP);
}

// dY (fp32, at the output of layer l whose output is Y, input X):
// dA = relu'(Y) dY (bf16); dskip += dA; weight grads; dX = conv^T(dA) (fp32)
static void layer_bwd(cb_net_s* N, int l, const float* dY, const u16* Y, const u16* X, float* dskip, float* dX, int n,
                      int H, int W, bool relu = true) {
  const long long cnt = (long long)n * H * W * C;
  if (relu) hipLaunchKernelGGL(k_relu_bwd, egrid(cnt), dim3(256), 0, N->stream, dY, Y, N->ga, dskip, cnt);
  else hipLaunchKernelGGL(k_to_bf16, egrid(cnt), dim3(256), 0, N->stream, dY, N->ga, cnt);
  wgrad(N, l, N->ga, X, n, H, W);
  if (dX) conv(N, l, N->ga, nullptr, false, nullptr, dX, n, H, W, true);
}

static void backward(cb_net_s* N, int n) {
  const int H = N->H, W = N->W;
  // head: dY in g0 (channel 0 = dz)
  layer_bwd(N, 11, N->g0, nullptr, N->e[0], nullptr, N->g1, n, H, W, false);  // g1 = d e0
  for (int l = 0; l < 4; l++)
    hipLaunchKernelGGL(k_zero, egrid((long long)n * (H >> l) * (W >> l) * C), dim3(256), 0, N->stream, N->gs[l],
                       (long long)n * (H >> l) * (W >> l) * C);
  // decoder, l = 0, 1, 2: e[l] = relu(conv(up[l]) + s[l]); d e[l] in cur
  float* cur = N->g1;
  float* other = N->g0;
  for (int l = 0; l < 3; l++) {
    const int h = H >> l, w = W >> l;
    layer_bwd(N, 10 - l, cur, N->e[l], N->up[l], N->gs[l], other, n, h, w);  // other = d up[l]
    // d e[l+1] (d s3 after the last decoder layer) = up_bwd(d up[l])
    float* dst = l < 2 ? cur : N->gs[3];
    hipLaunchKernelGGL(k_up_bwd, egrid((long long)n * (h / 2) * (w / 2) * C), dim3(256), 0, N->stream, other, dst, n,
                       h / 2, w / 2);
  }
  // encoder, deepest first: s[l] = relu(conv(h[l])), h[l] = relu(conv(in_l))
  for (int l = 3; l >= 0; l--) {
    const int h = H >> l, w = W >> l;
    layer_bwd(N, 2 * l + 1, N->gs[l], N->s[l], N->h[l], nullptr, N->g0, n, h, w);  // g0 = d h[l]
    const u16* in = l > 0 ? N->pin[l] : N->x0;
    layer_bwd(N, 2 * l, N->g0, N->h[l], in, nullptr, l > 0 ? N->g1 : nullptr, n, h, w);  // g1 = d pin[l]
    if (l > 0)
      hipLaunchKernelGGL(k_pool_bwd, egrid((long long)n * 2 * h * 2 * w * C), dim3(256), 0, N->stream, N->g1,
                         N->gs[l - 1], n, 2 * h, 2 * w);
  }
}

extern "C" int cb_net_forward(cb_net N, int n, const float* x, float* z16) {
  if (!N || !x) return cb_fail(CB_E_INVALID, "null argument");
  if (n < 1 || n > N->batch) return cb_fail(CB_E_INVALID, "batch size out of range");
  const long long cnt = (long long)n * N->H * N->W * C;
  hipLaunchKernelGGL(k_to_bf16, egrid(cnt), dim3(256), 0, N->stream, x, N->x0, cnt);
  forward(N, n);
  if (z16) CB_HIP(hipMemcpyAsync(z16, N->head, cnt * 4, hipMemcpyDeviceToDevice, N->stream));
  CB_HIP(hipGetLastError());
  return CB_OK;
}

extern "C" int cb_net_loss_grad(cb_net N, int n, const float* x, const float* t, double* loss_host, float* grad) {
  if (!N || !x || !t) return cb_fail(CB_E_INVALID, "null argument");
  if (int rc = cb_net_forward(N, n, x, nullptr)) return rc;
  const int HW = N->H * N->W;
  hipLaunchKernelGGL(k_head_loss, dim3(n), dim3(256), 0, N->stream, N->head, t, N->g0, N->lossv, HW, n);
  backward(N, n);
  CB_HIP(hipMemcpyAsync(N->lossh, N->lossv, n * 8, hipMemcpyDeviceToHost, N->stream));
  if (grad) CB_HIP(hipMemcpyAsync(grad, N->grad, NPARAM * 4, hipMemcpyDeviceToDevice, N->stream));
  CB_HIP(hipStreamSynchronize(N->stream));
  if (loss_host) {
    double s = 0.0;
    for (int i = 0; i < n; i++) s += N->lossh[i];
    *loss_host = s / n;
  }
  return CB_OK;
}

extern "C" int cb_net_adam_step(cb_net N, float lr) {
  if (!N) return cb_fail(CB_E_INVALID, "null net");
  N->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)N->step), c2 = 1.f - powf(b2, (float)N->step);
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, N->stream, N->prm, N->grad, N->m1, N->m2, lr,
                     b1, b2, 1e-8f, c1, c2);
  hipLaunchKernelGGL(k_weights_bf16, dim3((NLAYER * LW + 255) / 256), dim3(256), 0, N->stream, N->prm, N->wf, N->wb);
  CB_HIP(hipGetLastError());
  return CB_OK;
}

// One problem of a warm-start launch: argument checks and the scalars of
// its features (f: N x N profile, x: its G x G x C feature block).
static int ws_problem(cb_net N, const double* f, int Nf, double L, double h, double E1, double nu1, double E2,
                      double nu2, double F, float* x, WsProblem* q) {
  if (!N || !f || !x) return cb_fail(CB_E_INVALID, "null argument");
  if (!cb::aligned16(f)) return cb_fail(CB_E_INVALID, "f must be 16-byte aligned");
  if (N->H != N->W) return cb_fail(CB_E_INVALID, "square net grid required");
  const int G = N->H;
  if (Nf < 8 || (Nf % G != 0 && G % Nf != 0)) return cb_fail(CB_E_INVALID, "N must divide or be a multiple of the net grid");
  const double E2s = E2 / (1.0 - nu2 * nu2);
  *q = WsProblem{};
  q->f = f;
  q->x = x;
  q->N = Nf;
  q->L = L;
  q->sc.s[0] = (float)(std::log10(std::max(h, 1e-12) / L) / 3.0);
  q->sc.s[1] = (float)(std::log10(E1 / E2) / 2.0);
  q->sc.s[2] = (float)(2.0 * nu1);
  q->sc.s[3] = (float)(2.0 * nu2);
  q->sc.s[4] = (float)(std::log10(std::max(F, 1e-300) / (E2s * L * L)) / 4.0);
  q->sc.s[5] = 1.f;
  return CB_OK;
}

// features of the nq problems of B (slots base ..): min f, then the features
static void ws_features(cb_net N, const WsBatch& B, int base, int nq) {
  hipLaunchKernelGGL(k_fmin, dim3(RP, nq), dim3(256), 0, N->stream, B, base, N->scratch);
  hipLaunchKernelGGL(k_features, dim3(egrid((long long)N->H * N->H).x, nq), dim3(256), 0, N->stream, B, base, N->H,
                     (const double*)N->scratch);
}

extern "C" int cb_net_features(cb_net N, const double* f, int Nf, double L, double h, double E1, double nu1, double E2,
                               double nu2, double F, float* x) {
  WsBatch B{};
  if (int rc = ws_problem(N, f, Nf, L, h, E1, nu1, E2, nu2, F, x, &B.q[0])) return rc;
  ws_features(N, B, 0, 1);
  CB_HIP(hipGetLastError());
  return CB_OK;
}

extern "C" int cb_net_warmstart_batch(cb_net N, int n, const cb_plan* plans, const double* const* f,
                                      const double* F_host, double cut, double* const* p_out) {
  if (!N || !plans || !f || !F_host || !p_out) return cb_fail(CB_E_INVALID, "null argument");
  if (n < 1 || n > N->batch) return cb_fail(CB_E_INVALID, "batch size out of range");
  if (!(cut >= 0.0)) return cb_fail(CB_E_INVALID, "cut must be >= 0");
  const size_t hwc = (size_t)N->H * N->W * C;
  // problems in launches of up to WS_MAX (problem index in the batch = base + q)
  std::vector<WsBatch> groups((n + WS_MAX - 1) / WS_MAX);
  int maxN = 0;
  for (int i = 0; i < n; i++) {
    const cb_plan P = plans[i];
    if (!P || !f[i] || !p_out[i]) return cb_fail(CB_E_INVALID, "null plan or array in the batch");
    WsProblem& q = groups[i / WS_MAX].q[i % WS_MAX];
    if (int rc = ws_problem(N, f[i], P->N, P->L, P->h, P->E1, P->nu1, P->E2, P->nu2, F_host[i], N->feat + i * hwc, &q))
      return rc;
    q.p = p_out[i];
    // stiff thin coating: no guess (zeros; the solve then takes its cold
    // start): the network's guess measured slower than a cold start there.
    // Layered stacks and periodic plans lie outside its training data.
    q.guess = !(P->precond_auto == 1 || P->layered || P->kernel_mode != CB_KERNEL_PADDED);
    maxN = std::max(maxN, P->N);
  }
  for (size_t g = 0; g < groups.size(); g++)
    ws_features(N, groups[g], (int)g * WS_MAX, std::min(WS_MAX, n - (int)g * WS_MAX));
  if (int rc = cb_net_forward(N, n, N->feat, nullptr)) return rc;
  double* mean = N->scratch + (size_t)N->batch * RP;
  for (size_t g = 0; g < groups.size(); g++) {
    const int base = (int)g * WS_MAX, nq = std::min(WS_MAX, n - base);
    hipLaunchKernelGGL(k_qmean, dim3(RP, nq), dim3(256), 0, N->stream, groups[g], base, (const float*)N->head, N->H,
                       mean, N->sp);
    hipLaunchKernelGGL(k_prolong, dim3(egrid((long long)maxN * maxN).x, nq), dim3(256), 0, N->stream, groups[g], base,
                       (const float*)N->sp, N->H, (const double*)mean, cut);
  }
  CB_HIP(hipGetLastError());
  CB_HIP(hipStreamSynchronize(N->stream));
  return CB_OK;
}

extern "C" int cb_net_warmstart(cb_net N, cb_plan P, const double* f, double F, double cut, double* p_out) {
  return cb_net_warmstart_batch(N, 1, &P, &f, &F, cut, &p_out);
}
