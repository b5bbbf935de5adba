// cb_apply_K_noalloc: the zero-padded FFT convolution u = K p (Eq. 1
// evaluated as Eq. 11) without a plan and without any device allocation.
//
// The half-spectrum intermediate of the three transforms lives in the
// file-scope device array `scratch` below instead of plan-owned memory.
// Each device holds its own copy of the array (from module load until the
// process ends) at its own address: the host looks that address up once
// per device with hipGetSymbolAddress and passes it to the kernels.  In
// host code the array's name is only a host-side stand-in and is never
// passed to a kernel or a copy.
//
// Every call on one device shares that device's array: calls that overlap
// in time on one device (two streams, two threads) race on it, and the
// caller must order them.  The kernels overwrite every element they read
// before reading it, so nothing needs clearing between calls.
#include <mutex>

#include "internal.h"

namespace cb {
namespace {

// Largest grid served: N = 1024 in FP64 (N (N + 1) complex doubles,
// 16.8 MB); FP32 uses half of it per cell.
constexpr int NOALLOC_NMAX = 1024;
constexpr size_t NOALLOC_BYTES = (size_t)NOALLOC_NMAX * (NOALLOC_NMAX + 1) * 16;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::once_flag g_once[MAX_DEVICES];
void* g_scratch[MAX_DEVICES] = {};
hipError_t g_init_err[MAX_DEVICES] = {};

// Once per device, with that device current: the device address of its
// `scratch`, and the dynamic-LDS attributes of the convolution kernels of
// every size served (so no attribute is set while a caller captures).
void init_device(int dev) {
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr == nullptr) e = hipErrorInvalidSymbol;
  if (e == hipSuccess)
    for (int lg = 4; (1 << lg) <= NOALLOC_NMAX; lg++) prepare_apply(lg);
  g_init_err[dev] = e;
  g_scratch[dev] = e == hipSuccess ? ptr : nullptr;
}

}  // namespace
}  // namespace cb

extern "C" int cb_apply_K_noalloc(int N, int precision, const void* table, const void* p, void* u, void* stream) {
  using namespace cb;
  if (N < 16 || N > NOALLOC_NMAX || (N & (N - 1)))
    return cb_fail_c(CB_E_INVALID, "cb_apply_K_noalloc: N must be a power of two in [16, 1024] "
                                   "(the static scratch holds the N = 1024 FP64 intermediate)");
  if (precision != CB_FP64 && precision != CB_FP32)
    return cb_fail_c(CB_E_INVALID, "cb_apply_K_noalloc: precision must be CB_FP64 or CB_FP32");
  if (!table || !p || !u) return cb_fail_c(CB_E_INVALID, "cb_apply_K_noalloc: null array");
  if (p == u) return cb_fail_c(CB_E_INVALID, "cb_apply_K_noalloc: u must not alias p");
  if (!aligned16(table) || !aligned16(p) || !aligned16(u))
    return cb_fail_c(CB_E_INVALID, "cb_apply_K_noalloc: table, p and u must be 16-byte aligned");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return cb_fail_c(CB_E_DEVICE, "cb_apply_K_noalloc: no usable current device");
  std::call_once(g_once[dev], init_device, dev);
  if (g_init_err[dev] != hipSuccess)
    return cb_fail_c(CB_E_DEVICE, "cb_apply_K_noalloc: hipGetSymbolAddress of the scratch array failed");
  // a stack plan that points at the caller's table and the device scratch
  // (no tables, workspace or streams of its own); default launch shape
  cb_plan_s P;
  P.N = N;
  P.M = 2 * N;
  while ((1 << P.log2n) < N) P.log2n++;
  P.precision = precision;
  P.d_table = const_cast<void*>(table);
  P.d_S = g_scratch[dev];
  P.device = dev;
  const hipError_t e = launch_apply(&P, p, u, (hipStream_t)stream);
  if (e != hipSuccess) return cb_fail_c(CB_E_DEVICE, hipGetErrorString(e));
  return CB_OK;
}
