// Device building blocks for the zero-padded real 2-D FFT convolution.
//
// Stockham autosort passes over lines held in LDS, radix 2..16 butterflies
// in registers, twiddles from a two-level table (64-entry fine table times
// a coarse table) so that every twiddle is one complex product of two
// correctly rounded values.  All sizes are compile-time constants.
#pragma once
#include <hip/hip_runtime.h>

namespace cb {

template <typename T> struct cx_of;
template <> struct cx_of<float> { using type = float2; };
template <> struct cx_of<double> { using type = double2; };
template <typename T> using cx = typename cx_of<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { return C{a.x * s, a.y * s}; }
// a * (-i) for the forward direction (DIR = +1), a * (+i) for the inverse.
template <int DIR, typename C> __device__ __forceinline__ C mul_mi(C a) {
  if constexpr (DIR > 0) return C{a.y, -a.x};
  else return C{-a.y, a.x};
}

// exp(-DIR * 2 pi i m / 16) for m in [1, 8), as exact-to-rounding constants.
template <typename T, int DIR>
__device__ __forceinline__ cx<T> root16(int m) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
  constexpr double c2 = 0.70710678118654752440;
  double c = 1.0, s = 0.0;
  switch (m) {
    case 1: c = c1; s = s1; break;
    case 2: c = c2; s = c2; break;
    case 3: c = s1; s = c1; break;
    case 4: c = 0.0; s = 1.0; break;
    case 5: c = -s1; s = c1; break;
    case 6: c = -c2; s = c2; break;
    case 7: c = -c1; s = s1; break;
    default: break;
  }
  return cx<T>{T(c), T(DIR > 0 ? -s : s)};
}

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
  return r;
}

// In-register DFT of length R (power of two, <= 16), natural order in and
// out.  DIR = +1: sum a_n exp(-2 pi i n k / R); DIR = -1: exp(+...).
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft(cx<T>* a) {
  using C = cx<T>;
#pragma unroll
  for (int i = 0; i < R; i++) {
    const int j = bitrev<R>(i);
    if (j > i) { C t = a[i]; a[i] = a[j]; a[j] = t; }
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; k++) {
        C v = a[i + k + len / 2];
        const int m = k * (16 / len);
        if (m == 4) v = mul_mi<DIR>(v);
        else if (m != 0) v = cmul(v, root16<T, DIR>(m));
        const C u = a[i + k];
        a[i + k] = cadd(u, v);
        a[i + k + len / 2] = csub(u, v);
      }
    }
  }
}

// x * exp(-DIR 2 pi i n / R) for 0 <= n < R/2, R <= 16 (a constant root).
template <typename T, int R, int DIR>
__device__ __forceinline__ cx<T> rot_root(cx<T> x, int n) {
  const int m = n * (16 / R);
  if (m == 0) return x;
  if (m == 4) return mul_mi<DIR>(x);
  return cmul(x, root16<T, DIR>(m));
}

// DFT of length R whose upper half of inputs a[R/2..R-1] is zero (not
// read): X[2m] is the length-R/2 DFT of a, X[2m+1] that of a[n] w^n.
// Natural-order outputs in a[0..R-1].
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_half_in(cx<T>* a) {
  using C = cx<T>;
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    a[1] = a[0];
  } else {
    constexpr int H = R / 2;
    C e[H], o[H];
#pragma unroll
    for (int n = 0; n < H; n++) {
      e[n] = a[n];
      o[n] = rot_root<T, R, DIR>(a[n], n);
    }
    dft<T, H, DIR>(e);
    dft<T, H, DIR>(o);
#pragma unroll
    for (int m = 0; m < H; m++) {
      a[2 * m] = e[m];
      a[2 * m + 1] = o[m];
    }
  }
}

// DFT of length R of which only the lower half of the outputs is formed:
// X[k] = E[k] + w^k O[k], k < R/2, E and O the length-R/2 DFTs of the even
// and odd inputs; written to a[0..R/2-1] (the upper half is left undefined).
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_half_out(cx<T>* a) {
  using C = cx<T>;
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    a[0] = cadd(a[0], a[1]);
  } else {
    constexpr int H = R / 2;
    C e[H], o[H];
#pragma unroll
    for (int n = 0; n < H; n++) {
      e[n] = a[2 * n];
      o[n] = a[2 * n + 1];
    }
    dft<T, H, DIR>(e);
    dft<T, H, DIR>(o);
#pragma unroll
    for (int k = 0; k < H; k++) a[k] = cadd(e[k], rot_root<T, R, DIR>(o[k], k));
  }
}

// Two-level twiddle table for a transform length LT (power of two):
// w(e) = exp(-2 pi i e / LT) = hi[e >> 6] * lo[e & 63] (LT > 64), lo[e] else.
template <typename T, int LT>
struct Tw {
  static constexpr int NLO = LT < 64 ? LT : 64;
  static constexpr int NHI = LT <= 64 ? 1 : LT / 64;
  const cx<T>* lo;
  const cx<T>* hi;
  __device__ __forceinline__ cx<T> get(int e) const {
    if constexpr (LT <= 64) return lo[e];
    else return cmul(hi[e >> 6], lo[e & 63]);
  }
  // cooperative evaluation of both tables into LDS (lo then hi), in FP64
  // (sincospi of an exact binary fraction) rounded once to T
  __device__ __forceinline__ static void compute(cx<T>* dst, int tid, int nthreads) {
    for (int i = tid; i < NLO + NHI; i += nthreads) {
      const int e = i < NLO ? i : 64 * (i - NLO);
      double s, c;
      sincospi(2.0 * (double)e / (double)LT, &s, &c);
      dst[i] = cx<T>{T(c), T(-s)};
    }
  }
};

// LDS padding: one extra slot every 2^PS elements.
template <int PS>
__device__ __forceinline__ int padi(int i) { return i + (i >> PS); }
template <int PS>
__host__ __device__ constexpr int padded(int n) { return n + (n >> PS) + 1; }

// Radix used by the pass at stride Ls for a length-L line with E elements
// per thread.
__host__ __device__ constexpr int pick_radix(int L, int E, int Ls) {
  int r = E < 16 ? E : 16;
  return (L / Ls) < r ? (L / Ls) : r;
}
// Radix of the last pass of the greedy schedule that starts at stride Ls0.
__host__ __device__ constexpr int last_radix_from(int L, int E, int Ls0) {
  int Ls = Ls0, r = 1;
  while (Ls < L) { r = pick_radix(L, E, Ls); Ls *= r; }
  return r;
}
__host__ __device__ constexpr int last_radix(int L, int E) { return last_radix_from(L, E, 1); }

// The R - 1 twiddles w^i, w = exp(-2 pi i k scale / LT), of butterfly j of
// a Stockham pass at stride Ls > 1 (k = j mod Ls, scale = LT / (Ls R)),
// into w[1..R-1].  They come from table lookups of w, w^4 and (R = 16) w^8
// and products of at most two further factors, so that each is within a
// few roundings of exact while most lookups (two LDS reads, index
// arithmetic and a product each) are saved.
template <typename T, int LT, int R, int Ls>
__device__ __forceinline__ void twiddles(cx<T>* w, int j, const Tw<T, LT>& tw) {
  const int k = j & (Ls - 1);
  constexpr int scale = LT / (Ls * R);
  if constexpr (R <= 4) {
#pragma unroll
    for (int i = 1; i < R; i++) w[i] = tw.get(i * k * scale);
  } else {
    const int e = k * scale;
    w[1] = tw.get(e);
    w[4] = tw.get(4 * e);
    w[2] = cmul(w[1], w[1]);
    w[3] = cmul(w[2], w[1]);
#pragma unroll
    for (int i = 5; i < 8; i++) w[i] = cmul(w[4], w[i - 4]);
    if constexpr (R == 16) {
      w[8] = tw.get(8 * e);
      w[12] = cmul(w[8], w[4]);
#pragma unroll
      for (int i = 9; i < 12; i++) w[i] = cmul(w[8], w[i - 8]);
#pragma unroll
      for (int i = 13; i < 16; i++) w[i] = cmul(w[12], w[i - 12]);
    }
  }
}

// Twiddle then DFT of one butterfly of a Stockham pass (stride Ls, radix R,
// twiddle-table length LT, line length L; j = butterfly index).
// HALF_OUT: only the lower half of the butterfly's outputs is formed.
template <typename T, int L, int LT, int R, int Ls, int DIR, bool HALF_OUT = false>
__device__ __forceinline__ void butterfly(cx<T>* a, int j, const Tw<T, LT>& tw) {
  if constexpr (Ls > 1) {
    cx<T> w[R];
    twiddles<T, LT, R, Ls>(w, j, tw);
#pragma unroll
    for (int i = 1; i < R; i++) {
      if constexpr (DIR < 0) w[i].y = -w[i].y;
      a[i] = cmul(a[i], w[i]);
    }
  }
  if constexpr (HALF_OUT) dft_half_out<T, R, DIR>(a);
  else dft<T, R, DIR>(a);
}

// The conjugate transpose of a forward butterfly: inverse DFT, then the
// conjugated twiddles of the same butterfly.  Taking the forward passes in
// reverse order this way gives the inverse transform (each forward pass is
// a permutation, a diagonal of twiddles and DFTs; its conjugate transpose
// undoes it up to the factor R): the first pass, which has no twiddles,
// comes last.
template <typename T, int LT, int R, int Ls, bool HALF_OUT = false>
__device__ __forceinline__ void butterfly_t(cx<T>* a, int j, const Tw<T, LT>& tw) {
  if constexpr (HALF_OUT) dft_half_out<T, R, -1>(a);
  else dft<T, R, -1>(a);
  if constexpr (Ls > 1) {
    cx<T> w[R];
    twiddles<T, LT, R, Ls>(w, j, tw);
#pragma unroll
    for (int i = 1; i < (HALF_OUT ? R / 2 : R); i++) a[i] = cmul(a[i], cconj(w[i]));
  }
}

template <int R, int Ls>
__device__ __forceinline__ int out_index(int j, int i) {
  const int k = j & (Ls - 1);
  return (j - k) * R + k + i * Ls;
}

// One Stockham pass LDS -> LDS for the line at `buf` (NT threads, t).
// HOLD: the butterflies' twiddles are also left in wh[b * R + i] (one row
// of L / NT per pass) for the pass's conjugate transpose.
template <typename T, int L, int LT, int R, int Ls, int NT, int DIR, int PS, bool HOLD = false>
__device__ __forceinline__ void lds_pass(cx<T>* buf, int t, const Tw<T, LT>& tw, cx<T>* wh = nullptr) {
  constexpr int NB = L / (R * NT);
  cx<T> a[NB][R];
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int j = t + b * NT;
#pragma unroll
    for (int i = 0; i < R; i++) a[b][i] = buf[padi<PS>(j + i * (L / R))];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int j = t + b * NT;
    if constexpr (HOLD && Ls > 1) {
      cx<T> w[R];
      twiddles<T, LT, R, Ls>(w, j, tw);
#pragma unroll
      for (int i = 1; i < R; i++) {
        wh[b * R + i] = w[i];
        a[b][i] = cmul(a[b][i], DIR < 0 ? cconj(w[i]) : w[i]);
      }
      dft<T, R, DIR>(a[b]);
    } else {
      butterfly<T, L, LT, R, Ls, DIR>(a[b], j, tw);
    }
#pragma unroll
    for (int i = 0; i < R; i++) buf[padi<PS>(out_index<R, Ls>(j, i))] = a[b][i];
  }
  __syncthreads();
}

// The conjugate transpose of lds_pass at the same stride and radix: reads
// the forward pass's output positions, writes its input positions.  HOLD:
// the twiddles are the ones the forward pass (DIR = 1) left in wh.
template <typename T, int L, int LT, int R, int Ls, int NT, int PS, bool HOLD = false>
__device__ __forceinline__ void lds_pass_t(cx<T>* buf, int t, const Tw<T, LT>& tw, const cx<T>* wh = nullptr) {
  constexpr int NB = L / (R * NT);
  cx<T> a[NB][R];
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int j = t + b * NT;
#pragma unroll
    for (int i = 0; i < R; i++) a[b][i] = buf[padi<PS>(out_index<R, Ls>(j, i))];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int j = t + b * NT;
    if constexpr (HOLD && Ls > 1) {
      dft<T, R, -1>(a[b]);
#pragma unroll
      for (int i = 1; i < R; i++) a[b][i] = cmul(a[b][i], cconj(wh[b * R + i]));
    } else {
      butterfly_t<T, LT, R, Ls>(a[b], j, tw);
    }
#pragma unroll
    for (int i = 0; i < R; i++) buf[padi<PS>(j + i * (L / R))] = a[b][i];
  }
  __syncthreads();
}

// Number of passes with stride Ls0 <= Ls < LsEnd of a length-L line with E
// elements per thread.
__host__ __device__ constexpr int count_passes(int L, int E, int Ls0, int LsEnd) {
  int n = 0;
  for (int Ls = Ls0; Ls < LsEnd; Ls *= pick_radix(L, E, Ls)) n++;
  return n;
}

// All passes with stride Ls < LsEnd, LDS -> LDS.  HOLD: pass p leaves its
// twiddles in wh + p * (L / NT) (see lds_pass).
template <typename T, int L, int LT, int NT, int DIR, int PS, int Ls, int LsEnd, bool HOLD = false>
struct MidPasses {
  __device__ __forceinline__ static void run(cx<T>* buf, int t, const Tw<T, LT>& tw, cx<T>* wh = nullptr) {
    if constexpr (Ls < LsEnd) {
      constexpr int R = pick_radix(L, L / NT, Ls);
      lds_pass<T, L, LT, R, Ls, NT, DIR, PS, HOLD>(buf, t, tw, wh);
      MidPasses<T, L, LT, NT, DIR, PS, Ls * R, LsEnd, HOLD>::run(buf, t, tw, HOLD ? wh + L / NT : wh);
    }
  }
};

// The conjugate transposes of the passes MidPasses<..., Ls, LsEnd> runs, in
// reverse order (the inverse transform's middle passes); HOLD: with the
// twiddles MidPasses<..., 1, ..., HOLD> left in wh.
template <typename T, int L, int LT, int NT, int PS, int Ls, int LsEnd, bool HOLD = false>
struct MidPassesT {
  __device__ __forceinline__ static void run(cx<T>* buf, int t, const Tw<T, LT>& tw, const cx<T>* wh = nullptr) {
    if constexpr (Ls < LsEnd) {
      constexpr int R = pick_radix(L, L / NT, Ls);
      MidPassesT<T, L, LT, NT, PS, Ls * R, LsEnd, HOLD>::run(buf, t, tw, HOLD ? wh + L / NT : wh);
      lds_pass_t<T, L, LT, R, Ls, NT, PS, HOLD>(buf, t, tw, wh);
    }
  }
};

// XCD-aware block index: blocks are dealt round-robin to the 8 XCDs, so
// block b runs on XCD b % 8; hand each XCD a contiguous range of logical
// blocks so that neighbours sharing cache lines share an L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int per = (nblocks + 7) >> 3;
  const int xcd = b & 7;
  const int idx = b >> 3;
  // number of XCDs that receive `per` blocks vs `per - 1`
  const int full = nblocks - (per - 1) * 8;  // XCDs [0, full) get `per`
  int start = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
  return start + idx;
}

}  // namespace cb
