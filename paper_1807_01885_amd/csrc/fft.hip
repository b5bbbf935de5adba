// u = K p on the 2N-zero-padded grid (Eq. 1 evaluated as Eq. 11):
//
//   K1  rows, forward real FFT of length M = 2N of each of the N rows
//       (only the first N inputs non-zero), as a length-N complex FFT of
//       the packed pairs (x[2n] + i x[2n+1]) followed by the standard
//       even/odd split; writes the N+1 half-spectrum values of every row,
//       the two real ones (DC and Nyquist) packed into slot 0 as
//       X[0] + i X[N].
//   K2  columns, for each of the N half-spectrum columns (slot 0 carrying
//       the DC and Nyquist columns, separated around the multiply): forward complex
//       FFT of length M (first N inputs non-zero), multiply by the real
//       transfer table K^(|k|)/M^2, inverse FFT of length M, keep the first
//       N outputs.  The multiply sits between the last forward pass and the
//       first inverse pass, both register-resident.
//   K3  rows, inverse real FFT (Hermitian half spectrum, slot 0 unpacked,
//       -> first N of M real outputs).
//
// The same three kernels with PAD = false give the N-periodic convolution
// (real transforms of length N, no zero padding, N/2 + 1 half-spectrum
// columns): the solver's Fourier preconditioners are applied that way.
//
// Intermediate layout ("row tiles"): S[rb][kx][rr], rb = row / RB,
// rr = row % RB, kx in [0, N], complex; slot kx = N is allocated but
// unused.  K1/K3 read and write whole tiles (contiguous), K2 reads
// RB-element segments of a column.  With N + 1 columns one block of K2
// would be left over after an even share per CU; packing the two real
// columns removes it.
//
// This file is compiled once per launch-shape variant (CB_FFT_VARIANT =
// 0 .. CB_FFT_VARIANTS-1): elements per thread in K1/K3 and in K2 and the
// row-tile height differ, each variant lives in its own namespace, and the
// plan picks one (built-in default or the autotuner's choice).
#include <atomic>

#include "fft_core.h"
#include "internal.h"
#include "pk_dev.h"

#ifndef CB_FFT_VARIANT
#define CB_FFT_VARIANT 0
#endif
#define CB_CAT2(a, b) a##b
#define CB_CAT(a, b) CB_CAT2(a, b)

namespace cb {
namespace CB_CAT(fftv, CB_FFT_VARIANT) {

constexpr int VE1 = kFftVariants[CB_FFT_VARIANT].e_rows;
constexpr int VE2 = kFftVariants[CB_FFT_VARIANT].e_cols;
constexpr int VRBM = kFftVariants[CB_FFT_VARIANT].tile_mul;

constexpr int PS = 4;  // LDS padding shift

// ---------------------------------------------------------------------------
// K1: forward row transform
// ---------------------------------------------------------------------------
// PRO: the input EpiArgs `pro` mode PRO forms (0: p as given).
// `bid`: the block's index within its problem.
template <typename T, int LOG2N, bool PAD, int RB, int NT1, int G, int PRO = 0>
__device__ __forceinline__ void rows_fwd_body(int bid, const T* __restrict__ p, cx<T>* __restrict__ S,
                                              const int* __restrict__ skip, const EpiArgs& ea) {
  if (skip && (skip[0] | skip[1])) return;
  using C = cx<T>;
  // real transform length M, packed complex line L = M / 2
  constexpr int N = 1 << LOG2N, M = PAD ? 2 * N : N, L = M / 2, NC = L + 1;
  constexpr int ROWS = G * RB, NTH = ROWS * NT1, E = L / NT1;
  constexpr int LP = padded<PS>(L);
  using TW = Tw<T, M>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tws = reinterpret_cast<C*>(smem_raw);
  C* buf = tws + TW::NLO + TW::NHI;

  const int tid = threadIdx.x;
  const int lrow = tid / NT1, t = tid % NT1;
  const int row0 = bid * ROWS;
  C* line = buf + lrow * LP;

  // first pass (Ls = 1): packed inputs z[n], n < N/2, from global (with
  // padding the upper half of the line is zero); the loads are issued
  // before the twiddle tables are built
  {
    constexpr int R = pick_radix(L, E, 1);
    constexpr int NB = L / (R * NT1);
    const size_t rowoff = (size_t)(row0 + lrow) * N;
    const C* z = reinterpret_cast<const C*>(p + rowoff);
    // Formed inputs (PRO): the operands are loaded first, so that their
    // latency overlaps the folds of the partials that give the scalars
    // (every block folds them itself; the block-uniform return ends a
    // converged solve's iteration there).  Which x the direction takes
    // depends only on the phase.
    constexpr int RH = PAD ? R / 2 : R;  // pairs with data (upper half padding)
    const T* xs = nullptr;
    C* td = nullptr;  // t is read and rewritten through tdir (p is declared restrict)
    if constexpr (PRO == 1) {
      xs = static_cast<const T*>(ea.g);
    } else if constexpr (PRO == 2) {
      const bool pre = !(ea.plain0 && (!ea.two || ea.st->phase == 0));
      xs = static_cast<const T*>(pre ? ea.x : ea.g);
      td = reinterpret_cast<C*>(static_cast<T*>(ea.tdir) + rowoff);
    }
    uchar2 oa[NB][RH];
    C ox[NB][RH], ot[NB][RH];
    if constexpr (PRO != 0) {
#pragma unroll
      for (int b = 0; b < NB; b++) {
        const int j = t + b * NT1;
#pragma unroll
        for (int i = 0; i < RH; i++) {
          const int pi = j + i * (L / R);  // pair (cells 2 pi, 2 pi + 1 of the row)
          const size_t cell = rowoff + 2 * pi;
          oa[b][i] = *reinterpret_cast<const uchar2*>(ea.act + cell);
          ox[b][i] = *reinterpret_cast<const C*>(xs + cell);
          if constexpr (PRO == 2) ot[b][i] = td[pi];
        }
      }
    }
    double xbar = 0.0, beta = 0.0;
    if constexpr (PRO == 1) {
      if (!masked_gradient_scalars<NTH>(ea, xbar)) return;
    } else if constexpr (PRO == 2) {
      bool pre = false;
      if (!direction_scalars<NTH>(ea, xbar, beta, pre)) return;
    }
    C a[NB][R];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT1;
#pragma unroll
      for (int i = 0; i < R; i++) {
        if (i >= RH) {
          a[b][i] = C{T(0), T(0)};
          continue;
        }
        const int pi = j + i * (L / R);
        if constexpr (PRO == 0) {
          a[b][i] = z[pi];
        } else {
          const uchar2 a2 = oa[b][i];
          const C x2 = ox[b][i];
          if constexpr (PRO == 1) {
            a[b][i] = C{a2.x ? (T)((double)x2.x - xbar) : T(0), a2.y ? (T)((double)x2.y - xbar) : T(0)};
          } else {
            const C t2 = ot[b][i];
            const C tn = C{a2.x ? (T)(((double)x2.x - xbar) + beta * (double)t2.x) : T(0),
                           a2.y ? (T)(((double)x2.y - xbar) + beta * (double)t2.y) : T(0)};
            td[pi] = tn;
            a[b][i] = tn;
          }
        }
      }
    }
    TW::compute(tws, tid, NTH);
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT1;
      if constexpr (PAD) dft_half_in<T, R, 1>(a[b]);  // the upper half of the inputs is padding
      else dft<T, R, 1>(a[b]);
#pragma unroll
      for (int i = 0; i < R; i++) line[padi<PS>(out_index<R, 1>(j, i))] = a[b][i];
    }
    __syncthreads();
  }
  const TW tw{tws, tws + TW::NLO};
  MidPasses<T, L, M, NT1, 1, PS, pick_radix(L, E, 1), L>::run(line, t, tw);

  // split into the half spectrum of the length-M real transform:
  // X[k] = (Z[k] + conj Z[L-k])/2 - i/2 W^k (Z[k] - conj Z[L-k]),
  // W = exp(-2 pi i / M), k in [0, L].  One item forms the pair k, L - k,
  // which shares its two inputs and, as W^L = -1 (W^(L-k) = -conj W^k),
  // its twiddle; items in tile order (k major, rr minor), k in [0, L/2]
  constexpr int ITEMS = G * NC * RB;
  constexpr int PAIRS = L / 2 + 1;
  constexpr int PITEMS = G * PAIRS * RB;
  C* out = S + (size_t)bid * ITEMS;
#pragma unroll
  for (int it = 0; it < (PITEMS + NTH - 1) / NTH; it++) {
    const int q = tid + it * NTH;
    if (q < PITEMS) {
      const int g = q / (PAIRS * RB);
      const int qq = q - g * (PAIRS * RB);
      const int k = qq / RB;
      const int rr = qq - k * RB;
      const C* ln = buf + (g * RB + rr) * LP;
      C* o = out + g * (NC * RB) + rr;
      if (k == 0) {
        // X[0] and X[L] are real: both travel in slot 0 as X[0] + i X[L]
        // (slot L is left unwritten and K2 runs one column fewer)
        const C z0 = ln[padi<PS>(0)];
        o[0] = C{z0.x + z0.y, z0.x - z0.y};
      } else {
        const C zk = ln[padi<PS>(k)];
        const C zm = ln[padi<PS>(L - k)];
        const C w = tw.get(k);
        {
          const C zn = cconj(zm);
          const C e = cscale(cadd(zk, zn), T(0.5));
          const C od = cscale(csub(zk, zn), T(0.5));  // times -i below
          o[k * RB] = cadd(e, cmul(w, mul_mi<1>(od)));
        }
        if (k != L / 2) {
          const C zn = cconj(zk);
          const C e = cscale(cadd(zm, zn), T(0.5));
          const C od = cscale(csub(zm, zn), T(0.5));
          o[(L - k) * RB] = cadd(e, cmul(C{-w.x, w.y}, mul_mi<1>(od)));
        }
      }
    }
  }
}

template <typename T, int LOG2N, bool PAD, int RB, int NT1, int G, int PRO = 0>
__global__ void __launch_bounds__(G * RB * NT1)
k_rows_fwd(const T* __restrict__ p, cx<T>* __restrict__ S, const int* __restrict__ skip, EpiArgs ea) {
  rows_fwd_body<T, LOG2N, PAD, RB, NT1, G, PRO>(blockIdx.x, p, S, skip, ea);
}

// Several padded problems of one size in one launch: blocks
// [q nb, (q + 1) nb) transform problem q.
template <typename T, int LOG2N, int RB, int NT1, int G>
__global__ void __launch_bounds__(G * RB * NT1) k_rows_fwd_batch(ApplyBatch ba) {
  const int q = blockIdx.x / ba.nb;
  rows_fwd_body<T, LOG2N, true, RB, NT1, G, 0>(blockIdx.x - q * ba.nb, static_cast<const T*>(ba.p[q]),
                                                static_cast<cx<T>*>(ba.S[q]), nullptr, EpiArgs{});
}

// ---------------------------------------------------------------------------
// K2: column transform, transfer multiply, inverse column transform
// ---------------------------------------------------------------------------
// `tile`: the block's column tile within its problem.
template <typename T, int LOG2N, bool PAD, int RB, int NT2, int CB>
__device__ __forceinline__ void cols_body(int tile, cx<T>* __restrict__ S, const T* __restrict__ Tq,
                                          const int* __restrict__ skip) {
  if (skip && (skip[0] | skip[1])) return;
  using C = cx<T>;
  // NC half-spectrum columns; column 0 carries the DC and Nyquist columns
  // packed (X[0] + i X[M/2], both real), so NC - 1 columns are transformed
  constexpr int N = 1 << LOG2N, M = PAD ? 2 * N : N, L = M, NC = M / 2 + 1, NW = NC - 1;
  constexpr int NTH = CB * NT2, E = L / NT2;
  constexpr int LP = padded<PS>(L);
  constexpr int NBLK = (NW + CB - 1) / CB;
  using TW = Tw<T, M>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tws = reinterpret_cast<C*>(smem_raw);
  C* buf = tws + TW::NLO + TW::NHI;

  const int tid = threadIdx.x;
  const TW tw{tws, tws + TW::NLO};
  const int lc = tid / NT2, t = tid % NT2;
  const int kx = tile * CB + lc;
  const bool active = kx < NW;
  C* line = buf + lc * LP;

  constexpr int R0 = pick_radix(L, E, 1);
  constexpr int RL = last_radix(L, E);
  constexpr int NBL = L / (RL * NT2);
  // FP32: lanes past the last column transform column 0 and store nothing,
  // so that every load below is unconditional and the compiler issues them
  // together (a load under a branch ends in a wait of its own), and the
  // table values the multiply takes are loaded at the start.  FP64 keeps
  // the guarded first-pass loads and reads the table where it multiplies
  // (at N = 1024 K2 takes 12.5 us so, against 12.9 and 13.7 us with the
  // FP32 scheme or with the table loaded after the forward passes: the
  // registers are wanted by the forward passes).
  constexpr bool kEagerLoads = sizeof(T) == 4;
  // ... but not at radix-16 last passes (N = 2048, 4096), where the
  // prefetched row costs an occupancy step (N = 2048: 27.0 against 24.1 us)
  constexpr bool kPrefetchTable = kEagerLoads && RL <= 8;
  const int kxl = active ? kx : 0;
  const T* trow = Tq + (size_t)kxl * NC;
  T tq[NBL][RL];
  auto load_tq = [&]() {
#pragma unroll
    for (int b = 0; b < NBL; b++) {
#pragma unroll
      for (int i = 0; i < RL; i++) {
        const int ky = t + b * NT2 + i * (L / RL);
        tq[b][i] = trow[ky <= M / 2 ? ky : M - ky];
      }
    }
  };
  auto tval = [&](int b, int i) -> T {
    if constexpr (kPrefetchTable) {
      return tq[b][i];
    } else {
      const int ky = t + b * NT2 + i * (L / RL);
      return trow[ky <= M / 2 ? ky : M - ky];
    }
  };
  // forward first pass, inputs rows n < N from the tiles (upper half zero);
  // the loads are issued before the twiddle tables are built
  {
    constexpr int NB = L / (R0 * NT2);
    C a[NB][R0];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT2;
#pragma unroll
      for (int i = 0; i < R0; i++) {
        const int n = j + i * (L / R0);
        if constexpr (kEagerLoads)
          a[b][i] = (!PAD || i < R0 / 2) ? S[(size_t)(n / RB) * (NC * RB) + kxl * RB + (n % RB)] : C{T(0), T(0)};
        else
          a[b][i] = ((!PAD || i < R0 / 2) && active) ? S[(size_t)(n / RB) * (NC * RB) + kx * RB + (n % RB)]
                                                     : C{T(0), T(0)};
      }
    }
    if constexpr (kPrefetchTable) load_tq();
    TW::compute(tws, tid, NTH);
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT2;
      if constexpr (PAD) dft_half_in<T, R0, 1>(a[b]);  // rows N..M-1 are padding
      else dft<T, R0, 1>(a[b]);
#pragma unroll
      for (int i = 0; i < R0; i++) line[padi<PS>(out_index<R0, 1>(j, i))] = a[b][i];
    }
    __syncthreads();
  }
  // FP32 with a radix <= 8 last pass: each middle pass leaves its twiddles
  // in registers for its conjugate transpose (at most 32 complex values per
  // thread)
  constexpr int NMID = count_passes(L, E, R0, L / RL);
  constexpr bool kHoldTw = kPrefetchTable && NMID > 0 && NMID * E <= 32;
  C wh[kHoldTw ? NMID * E : 1];
  MidPasses<T, L, M, NT2, 1, PS, R0, L / RL, kHoldTw>::run(line, t, tw, wh);
  // last forward pass (stride L/RL) -> multiply -> first inverse pass, in registers
  {
    constexpr int NB = L / (RL * NT2);
    C a[NB][RL];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT2;
#pragma unroll
      for (int i = 0; i < RL; i++) a[b][i] = line[padi<PS>(j + i * (L / RL))];
    }
    __syncthreads();
    if (tile != 0) {
#pragma unroll
      for (int b = 0; b < NB; b++) {
        const int j = t + b * NT2;
        if constexpr (RL <= 8) {
          // the last forward pass and its conjugate transpose share the
          // butterfly's twiddles
          C w[RL];
          twiddles<T, M, RL, L / RL>(w, j, tw);
#pragma unroll
          for (int i = 1; i < RL; i++) a[b][i] = cmul(a[b][i], w[i]);
          dft<T, RL, 1>(a[b]);
#pragma unroll
          for (int i = 0; i < RL; i++) a[b][i] = cscale(a[b][i], tval(b, i));
          dft<T, RL, -1>(a[b]);
#pragma unroll
          for (int i = 1; i < RL; i++) a[b][i] = cmul(a[b][i], cconj(w[i]));
        } else {
          // radix 16: holding fifteen twiddles across the multiply costs an
          // occupancy step (N = 2048: FP64 K2 48.7 -> 74.7 us); form them twice
          butterfly<T, L, M, RL, L / RL, 1>(a[b], j, tw);
#pragma unroll
          for (int i = 0; i < RL; i++) a[b][i] = cscale(a[b][i], tval(b, i));
          butterfly_t<T, M, RL, L / RL>(a[b], j, tw);
        }
#pragma unroll
        for (int i = 0; i < RL; i++) line[padi<PS>(j + i * (L / RL))] = a[b][i];
      }
    } else {
      // the tile holding the packed column (block-uniform branch).  With
      // Z = C0 + i CN, C0 and CN the transforms of two real columns,
      // C0 = (Z[k] + conj Z[M-k]) / 2 and i CN = (Z[k] - conj Z[M-k]) / 2, so
      // T0 C0 + i TN CN = (T0 + TN)/2 Z[k] + (T0 - TN)/2 conj Z[M-k], whose
      // inverse is (T0 * x0) + i (TN * xN): both results stay packed.
      // FP32 loads the Nyquist row of the table together, before the
      // butterfly; FP64 reads it where it multiplies.
      const T* tn = Tq + (size_t)(NC - 1) * NC;
      T tnv[NB][RL];
      if constexpr (kPrefetchTable) {
#pragma unroll
        for (int b = 0; b < NB; b++) {
#pragma unroll
          for (int i = 0; i < RL; i++) {
            const int ky = t + b * NT2 + i * (L / RL);
            tnv[b][i] = tn[ky <= M / 2 ? ky : M - ky];
          }
        }
      }
#pragma unroll
      for (int b = 0; b < NB; b++) {
        const int j = t + b * NT2;
        butterfly<T, L, M, RL, L / RL, 1>(a[b], j, tw);
#pragma unroll
        for (int i = 0; i < RL; i++) line[padi<PS>(j + i * (L / RL))] = a[b][i];
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; b++) {
        const int j = t + b * NT2;
#pragma unroll
        for (int i = 0; i < RL; i++) {
          const int ky = j + i * (L / RL);
          if constexpr (kPrefetchTable) {
            const C zr = cconj(line[padi<PS>((L - ky) & (L - 1))]);
            const T t0 = tq[b][i], t1 = tnv[b][i];
            const C pk = cadd(cscale(a[b][i], T(0.5) * (t0 + t1)), cscale(zr, T(0.5) * (t0 - t1)));
            const C pl = cscale(a[b][i], t0);
            a[b][i] = kx == 0 ? pk : pl;
          } else {
            const int kq = ky <= M / 2 ? ky : M - ky;
            if (kx == 0) {
              const C zr = cconj(line[padi<PS>((L - ky) & (L - 1))]);
              const T t0 = trow[kq], t1 = tn[kq];
              a[b][i] = cadd(cscale(a[b][i], T(0.5) * (t0 + t1)), cscale(zr, T(0.5) * (t0 - t1)));
            } else {
              a[b][i] = cscale(a[b][i], trow[kq]);
            }
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; b++) {
        const int j = t + b * NT2;
        butterfly_t<T, M, RL, L / RL>(a[b], j, tw);
#pragma unroll
        for (int i = 0; i < RL; i++) line[padi<PS>(j + i * (L / RL))] = a[b][i];
      }
    }
    __syncthreads();
  }
  // inverse transform: the conjugate transposes of the forward passes in
  // reverse order (the last one is done above), so that the stride-1 pass,
  // which has no twiddles, comes last and writes the natural order
  MidPassesT<T, L, M, NT2, PS, R0, L / RL, kHoldTw>::run(line, t, tw, wh);
  {
    constexpr int NB = L / (R0 * NT2);
    C a[NB][R0];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT2;
#pragma unroll
      for (int i = 0; i < R0; i++) a[b][i] = line[padi<PS>(out_index<R0, 1>(j, i))];
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT2;
      butterfly_t<T, M, R0, 1, PAD>(a[b], j, tw);  // padded: only rows n < N are formed
      if (active) {
#pragma unroll
        for (int i = 0; i < (PAD ? R0 / 2 : R0); i++) {
          const int n = j + i * (L / R0);  // < N
          S[(size_t)(n / RB) * (NC * RB) + kx * RB + (n % RB)] = a[b][i];
        }
      }
    }
  }
}

// column tiles of one problem (the DC and Nyquist columns packed)
template <int LOG2N, bool PAD, int CB>
__host__ __device__ constexpr int col_tiles() {
  return (((PAD ? 2 : 1) << LOG2N) / 2 + CB - 1) / CB;
}

template <typename T, int LOG2N, bool PAD, int RB, int NT2, int CB>
__global__ void __launch_bounds__(CB * NT2)
k_cols(cx<T>* __restrict__ S, const T* __restrict__ Tq, const int* __restrict__ skip) {
  cols_body<T, LOG2N, PAD, RB, NT2, CB>(xcd_block(blockIdx.x, col_tiles<LOG2N, PAD, CB>()), S, Tq, skip);
}

// Several padded problems: the tiles of all problems are dealt to the XCDs
// as one range, so neighbouring tiles of a problem share an L2.
template <typename T, int LOG2N, int RB, int NT2, int CB>
__global__ void __launch_bounds__(CB * NT2) k_cols_batch(ApplyBatch ba) {
  constexpr int NB = col_tiles<LOG2N, true, CB>();
  const int g = xcd_block(blockIdx.x, NB * ba.n);
  const int q = g / NB;
  cols_body<T, LOG2N, true, RB, NT2, CB>(g - q * NB, static_cast<cx<T>*>(ba.S[q]), static_cast<const T*>(ba.T[q]),
                                        nullptr);
}

// ---------------------------------------------------------------------------
// K3: inverse row transform (half spectrum -> first N real outputs)
// ---------------------------------------------------------------------------
// EPI: the reduction of EpiArgs mode EPI (0: none) over the cells written.
template <typename T, int LOG2N, bool PAD, int RB, int NT1, int G, int EPI = 0>
__device__ __forceinline__ void rows_inv_body(int bid, const cx<T>* __restrict__ S, T* __restrict__ u,
                                              const int* __restrict__ skip, const EpiArgs& ea) {
  if (skip && (skip[0] | skip[1])) return;
  using C = cx<T>;
  constexpr int N = 1 << LOG2N, M = PAD ? 2 * N : N, L = M / 2, NC = L + 1;
  constexpr int ROWS = G * RB, NTH = ROWS * NT1, E = L / NT1;
  constexpr int LP = padded<PS>(L + 1);
  using TW = Tw<T, M>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tws = reinterpret_cast<C*>(smem_raw);
  C* buf = tws + TW::NLO + TW::NHI;

  const int tid = threadIdx.x;
  const TW tw{tws, tws + TW::NLO};
  constexpr int ITEMS = G * NC * RB;
  const C* in = S + (size_t)bid * ITEMS;
  // The operands of the EPI sums (the cells this thread writes in the last
  // pass) are loaded first, so that their latency overlaps the transform.
  constexpr int RL = last_radix(L, E);
  constexpr int NBL = L / (RL * NT1);
  constexpr int RHL = PAD ? RL / 2 : RL;  // outputs kept per butterfly
  const int lrow = tid / NT1, t = tid % NT1;
  const size_t row = (size_t)bid * ROWS + lrow;
  uchar2 e_act[NBL][RHL];
  C e_g[NBL][RHL], e_t[NBL][RHL];
  if constexpr (EPI != 0) {
#pragma unroll
    for (int b = 0; b < NBL; b++) {
#pragma unroll
      for (int i = 0; i < RHL; i++) {
        const size_t cell = row * N + 2 * (t + b * NT1 + i * (L / RL));
        e_act[b][i] = *reinterpret_cast<const uchar2*>(ea.act + cell);
        e_g[b][i] = *reinterpret_cast<const C*>(static_cast<const T*>(ea.g) + cell);
        if constexpr (EPI == 1) e_t[b][i] = *reinterpret_cast<const C*>(static_cast<const T*>(ea.t) + cell);
      }
    }
  }
  // Z[k] = (X[k] + conj X[L-k]) + i W^-k (X[k] - conj X[L-k]) for the pair
  // (k, L - k), read straight from the half spectrum (slot 0 holds
  // X[0] + i X[L], both real; slot L is unused); as W^L = -1 the pair shares
  // its twiddle.  Items in tile order (k major, rr minor), k in [0, L/2];
  // the loads are unconditional (the last items clamped) so that they are
  // issued together.
  constexpr int PAIRS = L / 2 + 1;
  constexpr int PITEMS = G * PAIRS * RB;
  constexpr int NIP = (PITEMS + NTH - 1) / NTH;
  {
    C xa[NIP], xb[NIP];
#pragma unroll
    for (int it = 0; it < NIP; it++) {
      const int q = tid + it * NTH;
      const int qc = q < PITEMS ? q : PITEMS - 1;
      const int g = qc / (PAIRS * RB);
      const int qq = qc - g * (PAIRS * RB);
      const int k = qq / RB;
      const int rr = qq - k * RB;
      const C* src = in + g * (NC * RB) + rr;
      xa[it] = src[k * RB];
      xb[it] = src[(L - k) * RB];
    }
    TW::compute(tws, tid, NTH);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIP; it++) {
      const int q = tid + it * NTH;
      if (q < PITEMS) {
        const int g = q / (PAIRS * RB);
        const int qq = q - g * (PAIRS * RB);
        const int k = qq / RB;
        const int rr = qq - k * RB;
        C* ln = buf + (g * RB + rr) * LP;
        const C xk = k == 0 ? C{xa[it].x, T(0)} : xa[it];
        const C xn = k == 0 ? C{xa[it].y, T(0)} : xb[it];
        const C w = cconj(tw.get(k));
        {
          const C sm = cadd(xk, cconj(xn));
          const C dd = csub(xk, cconj(xn));
          ln[padi<PS>(k)] = cadd(sm, mul_mi<-1>(cmul(w, dd)));
        }
        if (k != 0 && k != L / 2) {
          const C sm = cadd(xn, cconj(xk));
          const C dd = csub(xn, cconj(xk));
          ln[padi<PS>(L - k)] = cadd(sm, mul_mi<-1>(cmul(C{-w.x, w.y}, dd)));
        }
      }
    }
  }
  __syncthreads();
  C* line = buf + lrow * LP;
  MidPasses<T, L, M, NT1, -1, PS, 1, L / RL>::run(line, t, tw);
  {
    constexpr int NB = NBL;
    C* zo = reinterpret_cast<C*>(u + (size_t)(bid * ROWS + lrow) * N);
    C a[NB][RL];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT1;
#pragma unroll
      for (int i = 0; i < RL; i++) a[b][i] = line[padi<PS>(j + i * (L / RL))];
    }
    constexpr int Q = EPI == 1 ? 4 : 2;
    // the reduction below reuses the LDS: Q x NTH doubles
    static_assert(EPI == 0 || E >= 4, "row tile LDS too small for the K3 reductions");
    double v[Q] = {};
    double m = 0.0;
    if constexpr (EPI != 0) m = ea.st->gdev;
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = t + b * NT1;
      butterfly<T, L, M, RL, L / RL, -1, PAD>(a[b], j, tw);  // padded: only columns c < N are kept
#pragma unroll
      for (int i = 0; i < (PAD ? RL / 2 : RL); i++) {
        const int c = j + i * (L / RL);
        zo[c] = a[b][i];
        if constexpr (EPI != 0) {
          // cells 2c, 2c + 1 of this row: x = (a.x, a.y)
          const uchar2 a2 = e_act[b][i];
          const C g2 = e_g[b][i];
          const double x0 = (double)a[b][i].x, x1 = (double)a[b][i].y;
          const double g0 = (double)g2.x - m, g1 = (double)g2.y - m;
          if constexpr (EPI == 1) {
            const C t2 = e_t[b][i];
            const double t0 = (double)t2.x, t1 = (double)t2.y;
            if (a2.x) {
              v[0] += g0 * t0;
              v[1] += x0 * t0;
              v[2] += x0;
              v[3] += t0;
            }
            if (a2.y) {
              v[0] += g1 * t1;
              v[1] += x1 * t1;
              v[2] += x1;
              v[3] += t1;
            }
          } else {
            if (a2.x) {
              v[0] += x0;
              v[1] += g0 * x0;
            }
            if (a2.y) {
              v[0] += x1;
              v[1] += g1 * x1;
            }
          }
        }
      }
    }
    if constexpr (EPI != 0) {
      // fixed-order tree over the block, in the (now free) LDS
      double* red = reinterpret_cast<double*>(smem_raw);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; q++) red[q * NTH + tid] = v[q];
      __syncthreads();
      for (int h = NTH / 2; h > 0; h >>= 1) {
        if (tid < h) {
#pragma unroll
          for (int q = 0; q < Q; q++) red[q * NTH + tid] += red[q * NTH + tid + h];
        }
        __syncthreads();
      }
      if (tid == 0) {
#pragma unroll
        for (int q = 0; q < Q; q++) ea.region[8 + bid * Q + q] = red[q * NTH];
      }
    }
  }
}

template <typename T, int LOG2N, bool PAD, int RB, int NT1, int G, int EPI = 0>
__global__ void __launch_bounds__(G * RB * NT1)
k_rows_inv(const cx<T>* __restrict__ S, T* __restrict__ u, const int* __restrict__ skip, EpiArgs ea) {
  rows_inv_body<T, LOG2N, PAD, RB, NT1, G, EPI>(blockIdx.x, S, u, skip, ea);
}

template <typename T, int LOG2N, int RB, int NT1, int G>
__global__ void __launch_bounds__(G * RB * NT1) k_rows_inv_batch(ApplyBatch ba) {
  const int q = blockIdx.x / ba.nb;
  rows_inv_body<T, LOG2N, true, RB, NT1, G, 0>(blockIdx.x - q * ba.nb, static_cast<const cx<T>*>(ba.S[q]),
                                               static_cast<T*>(ba.u[q]), nullptr, EpiArgs{});
}

// ---------------------------------------------------------------------------
// launch shapes and dispatch
// ---------------------------------------------------------------------------
// PAD: the 2N-padded convolution of the operator; else the N-periodic one
template <int LOG2N, bool PAD = true> struct Shape {
  static constexpr int N = 1 << LOG2N, M = PAD ? 2 * N : N, L1 = M / 2;
  // the periodic lines are half as long: half the elements per thread
  // keeps the threads per line, and so the waves per launch (N = 1024,
  // tuned shape 3: FP32 19.4 -> 18.1 us, FP64 33.4 -> 31.2 us per
  // preconditioner application; mean over the six shapes FP32 21.7 ->
  // 18.7 us)
  static constexpr int VE1p = PAD ? VE1 : (VE1 / 2 < 4 ? 4 : VE1 / 2);
  static constexpr int VE2p = PAD ? VE2 : (VE2 / 2 < 4 ? 4 : VE2 / 2);
  static constexpr int E1 = L1 < VE1p ? L1 : VE1p;
  static constexpr int NT1 = L1 / E1;
  // the column kernel takes at least two passes (first and last differ)
  static constexpr int E2 = (PAD || VE2p <= M / 2) ? VE2p : M / 2;
  static constexpr int NT2 = M / E2;
  static constexpr int CB = NT2 >= 64 ? 1 : 64 / NT2;
};

template <typename T> constexpr int row_tile() { return (sizeof(T) == 4 ? 4 : 2) * VRBM; }

template <typename T, int LOG2N, bool PAD = true>
static size_t lds_rows(int G) {
  using SH = Shape<LOG2N, PAD>;
  using TW = Tw<T, SH::M>;
  return sizeof(cx<T>) * (TW::NLO + TW::NHI + (size_t)G * row_tile<T>() * padded<PS>(SH::L1 + 1));
}
template <typename T, int LOG2N, bool PAD = true>
static size_t lds_cols(int CB) {
  using SH = Shape<LOG2N, PAD>;
  using TW = Tw<T, SH::M>;
  return sizeof(cx<T>) * (TW::NLO + TW::NHI + (size_t)CB * padded<PS>(SH::M));
}

// row tiles per block of K1/K3: at least one wave of threads
template <typename T, int LOG2N, bool PAD = true>
constexpr int tiles_per_block() {
  using SH = Shape<LOG2N, PAD>;
  constexpr int RB = row_tile<T>();
  constexpr int G0 = (SH::NT1 * RB >= 64) ? 1 : 64 / (SH::NT1 * RB);
  return G0 > SH::N / RB ? SH::N / RB : G0;
}

// LDS bytes per block of the larger kernel; 0 if a block would exceed the
// 1024-thread limit (the shape is then not launchable at this size).  The
// periodic kernels of a size need no more threads or LDS than the padded.
template <typename T, int LOG2N>
static size_t lds_need() {
  using SH = Shape<LOG2N>;
  constexpr int G = tiles_per_block<T, LOG2N>();
  if (G * row_tile<T>() * SH::NT1 > 1024 || SH::CB * SH::NT2 > 1024) return 0;
  const size_t a = lds_rows<T, LOG2N>(G), b = lds_cols<T, LOG2N>(SH::CB);
  return a > b ? a : b;
}

template <typename T, int LOG2N, bool PAD>
static hipError_t apply_impl(int stages, const int* skip, const T* p, T* u, cx<T>* S, const T* Tq, const cx<T>* tw,
                             hipStream_t st, const EpiArgs* epi = nullptr) {
  using SH = Shape<LOG2N, PAD>;
  constexpr int N = SH::N, RB = row_tile<T>();
  constexpr int G = tiles_per_block<T, LOG2N, PAD>();
  constexpr int NC = SH::M / 2 + 1;
  const size_t lr = lds_rows<T, LOG2N, PAD>(G), lc = lds_cols<T, LOG2N, PAD>(SH::CB);
  auto k1 = k_rows_fwd<T, LOG2N, PAD, RB, SH::NT1, G>;
  auto k2 = k_cols<T, LOG2N, PAD, RB, SH::NT2, SH::CB>;
  auto k3 = k_rows_inv<T, LOG2N, PAD, RB, SH::NT1, G>;
  // the solver work the row transforms may carry: on the direction
  // convolution the direction update (K1, PRO 2) and the step sums (K3,
  // EPI 1); on the preconditioner convolution the masked gradient (K1,
  // PRO 1) and the sums of the preconditioned gradient (K3, EPI 2).  The
  // padded transforms only ever carry the direction; the periodic ones
  // carry either (periodic plans convolve their directions periodically).
  auto k1d = k_rows_fwd<T, LOG2N, PAD, RB, SH::NT1, G, 2>;
  auto k3d = k_rows_inv<T, LOG2N, PAD, RB, SH::NT1, G, 1>;
  auto k1p = k_rows_fwd<T, LOG2N, PAD, RB, SH::NT1, G, PAD ? 2 : 1>;
  auto k3p = k_rows_inv<T, LOG2N, PAD, RB, SH::NT1, G, PAD ? 1 : 2>;
  // set once per instantiation (plan creation calls this before any
  // capture; plans may be created on several threads, and setting the
  // attributes twice is harmless)
  static std::atomic<bool> attr{false};
  if (!attr.load(std::memory_order_acquire)) {
    hipFuncSetAttribute((const void*)k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    hipFuncSetAttribute((const void*)k1d, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    hipFuncSetAttribute((const void*)k1p, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lc);
    hipFuncSetAttribute((const void*)k3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    hipFuncSetAttribute((const void*)k3d, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    hipFuncSetAttribute((const void*)k3p, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    attr.store(true, std::memory_order_release);
  }
  const int nb_rows = N / (RB * G);
  const int nb_cols = (NC - 1 + SH::CB - 1) / SH::CB;  // DC and Nyquist columns packed
  if (epi && ((epi->mode != 0 && epi->mode != 1 && (PAD || epi->mode != 2)) ||
              (epi->pro != 0 && epi->pro != 2 && (PAD || epi->pro != 1))))
    return hipErrorInvalidValue;
  const dim3 grows(nb_rows), brows(G * RB * SH::NT1);
  if (stages & 1) {
    const int pro = epi ? epi->pro : 0;
    if (pro == 2) hipLaunchKernelGGL(k1d, grows, brows, lr, st, p, S, skip, *epi);
    else if (pro == 1) hipLaunchKernelGGL(k1p, grows, brows, lr, st, p, S, skip, *epi);
    else hipLaunchKernelGGL(k1, grows, brows, lr, st, p, S, skip, EpiArgs{});
  }
  if (stages & 2) hipLaunchKernelGGL(k2, dim3(nb_cols), dim3(SH::CB * SH::NT2), lc, st, S, Tq, skip);
  if (stages & 4) {
    const int mode = epi ? epi->mode : 0;
    if (mode == 1) hipLaunchKernelGGL(k3d, grows, brows, lr, st, (const cx<T>*)S, u, skip, *epi);
    else if (mode == 2) hipLaunchKernelGGL(k3p, grows, brows, lr, st, (const cx<T>*)S, u, skip, *epi);
    else hipLaunchKernelGGL(k3, grows, brows, lr, st, (const cx<T>*)S, u, skip, EpiArgs{});
  }
  return hipGetLastError();
}

// The padded convolution of ba.n problems: one launch per stage, the blocks
// of problem q after those of problems 0..q-1.  n = 0 only sets the
// kernels' dynamic-LDS attributes.
template <typename T, int LOG2N>
static hipError_t apply_batch_impl(const ApplyBatch& ba, hipStream_t st) {
  using SH = Shape<LOG2N, true>;
  constexpr int N = SH::N, RB = row_tile<T>();
  constexpr int G = tiles_per_block<T, LOG2N, true>();
  const size_t lr = lds_rows<T, LOG2N, true>(G), lc = lds_cols<T, LOG2N, true>(SH::CB);
  auto k1 = k_rows_fwd_batch<T, LOG2N, RB, SH::NT1, G>;
  auto k2 = k_cols_batch<T, LOG2N, RB, SH::NT2, SH::CB>;
  auto k3 = k_rows_inv_batch<T, LOG2N, RB, SH::NT1, G>;
  static std::atomic<bool> attr{false};
  if (!attr.load(std::memory_order_acquire)) {
    hipFuncSetAttribute((const void*)k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lc);
    hipFuncSetAttribute((const void*)k3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr);
    attr.store(true, std::memory_order_release);
  }
  if (ba.n <= 0) return hipSuccess;
  if (ba.n > CB_BATCH_MAX) return hipErrorInvalidValue;
  const int nb_rows = N / (RB * G);
  const int nb_cols = col_tiles<LOG2N, true, SH::CB>();
  ApplyBatch b = ba;
  b.nb = nb_rows;
  hipLaunchKernelGGL(k1, dim3(nb_rows * ba.n), dim3(G * RB * SH::NT1), lr, st, b);
  b.nb = nb_cols;
  hipLaunchKernelGGL(k2, dim3(nb_cols * ba.n), dim3(SH::CB * SH::NT2), lc, st, b);
  b.nb = nb_rows;
  hipLaunchKernelGGL(k3, dim3(nb_rows * ba.n), dim3(G * RB * SH::NT1), lr, st, b);
  return hipGetLastError();
}

template <typename T, int LOG2N, bool PAD>
constexpr int rows_blocks_n() {
  return (1 << LOG2N) / (row_tile<T>() * tiles_per_block<T, LOG2N, PAD>());
}

template <typename T, bool PAD>
static hipError_t apply_dispatch(int stages, const int* skip, int log2n, const T* p, T* u, cx<T>* S, const T* Tq,
                                 const cx<T>* tw, hipStream_t st, const EpiArgs* epi = nullptr) {
  switch (log2n) {
    case 4: return apply_impl<T, 4, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 5: return apply_impl<T, 5, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 6: return apply_impl<T, 6, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 7: return apply_impl<T, 7, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 8: return apply_impl<T, 8, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 9: return apply_impl<T, 9, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 10: return apply_impl<T, 10, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 11: return apply_impl<T, 11, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    case 12: return apply_impl<T, 12, PAD>(stages, skip, p, u, S, Tq, tw, st, epi);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t apply_any(bool periodic, int stages, const int* skip, int log2n, const T* p, T* u, cx<T>* S,
                            const T* Tq, hipStream_t st, const EpiArgs* epi) {
  return periodic ? apply_dispatch<T, false>(stages, skip, log2n, p, u, S, Tq, nullptr, st, epi)
                  : apply_dispatch<T, true>(stages, skip, log2n, p, u, S, Tq, nullptr, st, epi);
}

}  // namespace fftv<variant>

hipError_t CB_CAT(launch_apply_v, CB_FFT_VARIANT)(const cb_plan_s* P, const void* p, void* u, hipStream_t st,
                                                 int stages, const int* skip, const void* table, int prec,
                                                 const EpiArgs* epi) {
  using namespace CB_CAT(fftv, CB_FFT_VARIANT);
  // stages bit 3: the N-periodic convolution with the given table (the
  // preconditioners); a periodic plan's operator is N-periodic as well
  const bool given = (stages & 8) != 0;
  const bool periodic = given || P->kernel_mode == CB_KERNEL_PERIODIC;
  stages &= 7;
  if (given && !table) return hipErrorInvalidValue;
  if (prec == 0) {
    if (!table) table = P->precision == 0 ? P->d_table : P->d_table64;
    return apply_any<double>(periodic, stages, skip, P->log2n, (const double*)p, (double*)u, (cx<double>*)P->d_S,
                             (const double*)table, st, epi);
  }
  if (!table) table = P->d_table;
  return apply_any<float>(periodic, stages, skip, P->log2n, (const float*)p, (float*)u, (cx<float>*)P->d_S,
                          (const float*)table, st, epi);
}

// Set the dynamic-LDS attributes of every convolution kernel of this size
// (both precisions) up front, so that no attribute call happens while a
// stream is being captured.
namespace CB_CAT(fftv, CB_FFT_VARIANT) {
template <int LOG2N>
static void prepare_n() {
  float* nf = nullptr;
  double* nd = nullptr;
  (void)apply_impl<float, LOG2N, true>(0, nullptr, nf, nf, nullptr, nullptr, nullptr, nullptr);
  (void)apply_impl<double, LOG2N, true>(0, nullptr, nd, nd, nullptr, nullptr, nullptr, nullptr);
  (void)apply_impl<float, LOG2N, false>(0, nullptr, nf, nf, nullptr, nullptr, nullptr, nullptr);
  (void)apply_impl<double, LOG2N, false>(0, nullptr, nd, nd, nullptr, nullptr, nullptr, nullptr);
  (void)apply_batch_impl<float, LOG2N>(ApplyBatch{}, nullptr);
  (void)apply_batch_impl<double, LOG2N>(ApplyBatch{}, nullptr);
}
}  // namespace fftv<variant>

hipError_t CB_CAT(launch_apply_batch_v, CB_FFT_VARIANT)(int log2n, int prec, const ApplyBatch& ba, hipStream_t st) {
  using namespace CB_CAT(fftv, CB_FFT_VARIANT);
  switch (log2n) {
#define CB_BATCH_CASE(k) \
  case k: return prec == 0 ? apply_batch_impl<double, k>(ba, st) : apply_batch_impl<float, k>(ba, st);
    CB_BATCH_CASE(4) CB_BATCH_CASE(5) CB_BATCH_CASE(6) CB_BATCH_CASE(7)
    CB_BATCH_CASE(8) CB_BATCH_CASE(9) CB_BATCH_CASE(10) CB_BATCH_CASE(11) CB_BATCH_CASE(12)
#undef CB_BATCH_CASE
    default: return hipErrorInvalidValue;
  }
}

int CB_CAT(rows_blocks_v, CB_FFT_VARIANT)(int log2n, int prec, int periodic) {
  using namespace CB_CAT(fftv, CB_FFT_VARIANT);
  switch (log2n) {
#define CB_ROWS_CASE(k)                                                                               \
  case k:                                                                                             \
    return prec == 0 ? (periodic ? rows_blocks_n<double, k, false>() : rows_blocks_n<double, k, true>()) \
                     : (periodic ? rows_blocks_n<float, k, false>() : rows_blocks_n<float, k, true>());
    CB_ROWS_CASE(4) CB_ROWS_CASE(5) CB_ROWS_CASE(6) CB_ROWS_CASE(7)
    CB_ROWS_CASE(8) CB_ROWS_CASE(9) CB_ROWS_CASE(10) CB_ROWS_CASE(11) CB_ROWS_CASE(12)
#undef CB_ROWS_CASE
    default: return 0;
  }
}

size_t CB_CAT(lds_bytes_v, CB_FFT_VARIANT)(int log2n, int prec) {
  using namespace CB_CAT(fftv, CB_FFT_VARIANT);
  switch (log2n) {
#define CB_LDS_CASE(k) \
  case k: return prec == 0 ? lds_need<double, k>() : lds_need<float, k>();
    CB_LDS_CASE(4) CB_LDS_CASE(5) CB_LDS_CASE(6) CB_LDS_CASE(7)
    CB_LDS_CASE(8) CB_LDS_CASE(9) CB_LDS_CASE(10) CB_LDS_CASE(11) CB_LDS_CASE(12)
#undef CB_LDS_CASE
    default: return 0;
  }
}

void CB_CAT(prepare_apply_v, CB_FFT_VARIANT)(int log2n) {
  using namespace CB_CAT(fftv, CB_FFT_VARIANT);
  switch (log2n) {
    case 4: prepare_n<4>(); break;
    case 5: prepare_n<5>(); break;
    case 6: prepare_n<6>(); break;
    case 7: prepare_n<7>(); break;
    case 8: prepare_n<8>(); break;
    case 9: prepare_n<9>(); break;
    case 10: prepare_n<10>(); break;
    case 11: prepare_n<11>(); break;
    case 12: prepare_n<12>(); break;
    default: break;
  }
}

}  // namespace cb
