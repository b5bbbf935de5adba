// Convolution dispatch over the FFT launch-shape variants, and the
// autotuner that picks one per (device architecture, N, precision).
//
// The tuner times each variant as a graph of ten back-to-back convolutions
// on the plan's own stream (so host launch cost does not enter), replays it
// three times after one warm-up replay and keeps the fastest mean.  Tuned
// choices can be kept in a text cache, one line per entry:
//   <gcnArchName> <N> <precision 0|1> <variant index> <microseconds>
// The last matching line wins; the cache is only appended to.
#include <cmath>
#include <fstream>
#include <limits>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.h"

namespace cb {

using ApplyFn = hipError_t (*)(const cb_plan_s*, const void*, void*, hipStream_t, int, const int*, const void*, int,
                                const EpiArgs*);
static const ApplyFn kApply[CB_FFT_VARIANTS] = {launch_apply_v0, launch_apply_v1, launch_apply_v2,
                                                launch_apply_v3, launch_apply_v4, launch_apply_v5};
using RowsFn = int (*)(int, int, int);
static const RowsFn kRows[CB_FFT_VARIANTS] = {rows_blocks_v0, rows_blocks_v1, rows_blocks_v2,
                                              rows_blocks_v3, rows_blocks_v4, rows_blocks_v5};

hipError_t launch_apply(const cb_plan_s* P, const void* p, void* u, hipStream_t st, int stages, const int* skip,
                        const void* table, int prec, const EpiArgs* epi) {
  if (prec < 0) prec = P->precision;
  const int v = P->variant[prec == 0 ? 0 : 1];
  return kApply[v](P, p, u, st, stages, skip, table, prec, epi);
}

using BatchFn = hipError_t (*)(int, int, const ApplyBatch&, hipStream_t);
static const BatchFn kBatch[CB_FFT_VARIANTS] = {launch_apply_batch_v0, launch_apply_batch_v1, launch_apply_batch_v2,
                                                launch_apply_batch_v3, launch_apply_batch_v4, launch_apply_batch_v5};

hipError_t launch_apply_batch(const cb_plan_s* P0, const ApplyBatch& ba, hipStream_t st) {
  const int prec = P0->precision == CB_FP64 ? 0 : 1;
  return kBatch[P0->variant[prec]](P0->log2n, prec, ba, st);
}

int rows_blocks(const cb_plan_s* P, int prec, bool periodic) {
  if (prec < 0) prec = P->precision;
  const int v = P->variant[prec == 0 ? 0 : 1];
  return kRows[v](P->log2n, prec, periodic ? 1 : 0);
}

void prepare_apply(int log2n) {
  prepare_apply_v0(log2n);
  prepare_apply_v1(log2n);
  prepare_apply_v2(log2n);
  prepare_apply_v3(log2n);
  prepare_apply_v4(log2n);
  prepare_apply_v5(log2n);
  // a shape too large for the device's LDS fails its attribute call; that
  // shape is never launched (fft_variant_fits), so drop the error here
  // rather than let a later hipGetLastError report it
  (void)hipGetLastError();
}

using LdsFn = size_t (*)(int, int);
static const LdsFn kLds[CB_FFT_VARIANTS] = {lds_bytes_v0, lds_bytes_v1, lds_bytes_v2,
                                            lds_bytes_v3, lds_bytes_v4, lds_bytes_v5};

bool fft_variant_fits(int v, int log2n, int prec, int device) {
  int lim = 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return v == 0;
  const size_t need = kLds[v](log2n, prec);
  return need > 0 && need <= (size_t)lim;
}

static std::mutex g_cache_mu;

static bool cache_lookup(const char* path, const std::string& arch, int N, int prec, int* v, double* us) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ss(line);
    std::string a;
    int n = 0, pr = 0, vv = 0;
    double t = 0.0;
    if (ss >> a >> n >> pr >> vv >> t && a == arch && n == N && pr == prec && vv >= 0 && vv < CB_FFT_VARIANTS) {
      *v = vv;
      *us = t;
      found = true;
    }
  }
  return found;
}

static void cache_append(const char* path, const std::string& arch, int N, int prec, int v, double us) {
  std::ofstream out(path, std::ios::app);
  if (out) out << arch << ' ' << N << ' ' << prec << ' ' << v << ' ' << us << '\n';
}

// mean time of one convolution of precision prec (0 FP64, 1 FP32) with the
// plan's current variant for it, microseconds
static int time_variant(cb_plan_s* P, int prec, hipEvent_t e0, hipEvent_t e1, double* us) {
  constexpr int REPS = 10, REPLAYS = 3;
  hipStream_t st = P->istream;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipSuccess;
  {
    std::lock_guard<std::mutex> lk(graph_mutex());
    CB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < REPS && e == hipSuccess; r++)
      e = launch_apply(P, P->d_u, P->d_t, st, 7, nullptr, nullptr, prec);
    const hipError_t ee = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return cb_fail(CB_E_DEVICE, std::string("autotune capture: ") + hipGetErrorString(e != hipSuccess ? e : ee));
    }
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
  }
  if (e != hipSuccess) return cb_fail(CB_E_DEVICE, std::string("autotune instantiate: ") + hipGetErrorString(e));
  float ms = 0.f;
  e = hipGraphLaunch(ex, st);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < REPLAYS && e == hipSuccess; r++) e = hipGraphLaunch(ex, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (hipStreamSynchronize(st) != hipSuccess && e == hipSuccess) e = hipErrorUnknown;
  {
    std::lock_guard<std::mutex> lk(graph_mutex());
    (void)hipGraphExecDestroy(ex);
  }
  if (e != hipSuccess) return cb_fail(CB_E_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
  *us = 1000.0 * ms / (REPS * REPLAYS);
  return CB_OK;
}

// variant for one precision: from the cache, else timed (autotune = 1)
static int tune_one(cb_plan_s* P, int prec, int autotune, const char* cache, const std::string& arch, double* us_out) {
  *us_out = 0.0;
  if (cache) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int v = 0;
    double us = 0.0;
    if (cache_lookup(cache, arch, P->N, prec, &v, &us) && fft_variant_fits(v, P->log2n, prec, P->device)) {
      P->variant[prec] = v;
      *us_out = us;
      return CB_OK;
    }
  }
  if (!autotune) return CB_OK;
  // input p = 0 in d_u, output in d_t (both sized for FP64)
  CB_HIP(hipMemsetAsync(P->d_u, 0, (size_t)P->N * P->N * 8, P->istream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CB_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return cb_fail(CB_E_DEVICE, "event creation failed");
  }
  double best = std::numeric_limits<double>::infinity();
  int bestv = 0, rc = CB_OK;
  for (int v = 0; v < CB_FFT_VARIANTS && rc == CB_OK; v++) {
    if (!fft_variant_fits(v, P->log2n, prec, P->device)) continue;
    P->variant[prec] = v;
    double us = 0.0;
    rc = time_variant(P, prec, e0, e1, &us);
    if (rc == CB_OK && us < best) {
      best = us;
      bestv = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->variant[prec] = bestv;
  if (rc != CB_OK) return rc;
  *us_out = best;
  if (cache) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    cache_append(cache, arch, P->N, prec, bestv, best);
  }
  return CB_OK;
}

// The plan's precision, and for FP32 plans also the FP64 convolutions that
// refresh u = K p in the solvers.
int autotune_fft(cb_plan_s* P, int autotune, const char* cache) {
  if (!autotune && !cache) return CB_OK;
  hipDeviceProp_t prop;
  CB_HIP(hipGetDeviceProperties(&prop, P->device));
  const std::string arch = prop.gcnArchName;
  const int prec = P->precision == CB_FP64 ? 0 : 1;
  double us = 0.0, us64 = 0.0;
  if (int rc = tune_one(P, prec, autotune, cache, arch, &us)) return rc;
  P->tune_us = us;
  if (prec == 1)
    if (int rc = tune_one(P, 0, autotune, cache, arch, &us64)) return rc;
  return CB_OK;
}

}  // namespace cb
