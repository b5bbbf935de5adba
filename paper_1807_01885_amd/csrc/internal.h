// Internal plan state and launch entry points of libcoatbem.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/coatbem.h"

// Device-resident scalar state of one iterative solve.  Kernels read and
// write it so that a whole chunk of iterations runs without host traffic.
struct SolverState {
  double G_old;      // previous sum of squared gaps on the contact set
  double delta;      // 1: conjugate direction kept, 0: restart
  double tau;        // step length of the current iteration
  double d;          // rigid approach (prescribed, or found under force control)
  double gbar;       // mean gap on the contact set (force control)
  double rmean;      // mean of K t on the contact set (force control)
  double resid;      // relative residual of the last check
  double F;          // current total force
  double rr;         // masked CG: r.r
  double bnorm;      // masked CG: ||b||
  int done;          // 1 once converged (kernels of later iterations exit)
  int iters;         // iterations performed
  int nonfinite;     // 1 if a NaN/Inf was met
  int viol;          // penetrating cells outside the contact at last check
  int nactive;       // |Ic|
  int changed;       // adhesive: cells that changed state in the last round
  int pad[2];
};

struct cb_plan_s {
  int N = 0, M = 0, log2n = 0, precision = 0, dc_mode = 0;
  double L = 0, dx = 0, h = 0, E1 = 0, nu1 = 0, E2 = 0, nu2 = 0, dgamma = 0;
  double E1s = 0, E2s = 0, sigma_c = 0, k00 = 0, dc = 0;
  int validity_warning = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<double> table64;   // (N+1)^2, no 1/M^2
  // device memory owned by the plan
  void* d_table = nullptr;       // (N+1)^2, 1/M^2 folded, plan type
  void* d_tw = nullptr;          // twiddles lo|hi, plan complex type
  void* d_S = nullptr;           // N x (N+1) complex intermediate
  // solver workspace (plan type unless noted)
  void* d_u = nullptr;
  void* d_t = nullptr;
  void* d_r = nullptr;
  void* d_g = nullptr;
  void* d_pold = nullptr;
  unsigned char* d_mask = nullptr;   // scratch contact set (N*N)
  unsigned char* d_mask2 = nullptr;  // second contact-set buffer (N*N)
  unsigned char* d_det = nullptr;    // detached-in-this-step flags (N*N)
  double* d_part = nullptr;          // per-block FP64 partial sums
  SolverState* d_state = nullptr;
  SolverState* h_state = nullptr;    // pinned host mirror
  size_t workspace_bytes = 0;
  int nblk_red = 0;                  // blocks of the reduction kernels
};

namespace cb {
hipError_t launch_apply(const cb_plan_s* P, const void* p, void* u, hipStream_t st, int stages = 7);
size_t intermediate_elems(int N);
}  // namespace cb

// error reporting (thread-local message)
int cb_fail(int status, const std::string& msg);
#define CB_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return cb_fail(CB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
