// Batched solves: independent problems (uneven grids, materials, load modes)
// run concurrently, each on its own plan stream with its graph-captured
// iteration chunks.  A pool of host threads takes problems from a shared
// queue, the expected longest first; each thread drives one problem at a
// time, so up to `workers` problems keep the GPU busy while others wait on
// their convergence checks.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "internal.h"

extern "C" int cb_solve_batch(int n, const cb_plan* plans, const double* const* f, const double* target,
                              const int* mode, double* const* p_io, const cb_solve_opts* opts, int workers,
                              cb_result* out) {
  if (n < 0 || (n > 0 && (!plans || !f || !target || !mode || !p_io || !out)))
    return cb_fail(CB_E_INVALID, "null argument or negative count");
  if (n == 0) return CB_OK;
  std::set<const void*> seen;
  for (int i = 0; i < n; i++) {
    if (!plans[i] || !f[i] || !p_io[i]) return cb_fail(CB_E_INVALID, "null plan or array in the batch");
    if (mode[i] != 0 && mode[i] != 1) return cb_fail(CB_E_INVALID, "mode must be 0 (approach) or 1 (force)");
    if (!seen.insert(plans[i]).second) return cb_fail(CB_E_INVALID, "a plan appears twice in the batch");
  }
  int device = 0;
  CB_HIP(hipGetDevice(&device));
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  // Longest expected solve first, so that no long solve starts late and
  // runs alone at the end: larger grids first; within one grid, adhesive
  // approach steps (tens of detach/attach rounds), then stiff thin coatings
  // (the plans whose cold start takes the layer preconditioner; their
  // iteration count grows with the stiffness ratio E1*/E2*), then the rest
  // in the caller's order.
  auto rank = [&](int i) {
    const cb_plan_s* P = plans[i];
    const int cls = (mode[i] == 0 && P->dgamma > 0.0) ? 2 : (P->precond_auto == 1 ? 1 : 0);
    return std::make_tuple((long long)P->N * P->N, cls, cls == 1 ? P->E1s / P->E2s : 0.0);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rank(a) > rank(b); });
  // 16 by default: the N = 1024 force set gives 547 / 555 / 573 / 587 / 598 /
  // 607 solves/s at 3 / 4 / 6 / 8 / 12 / 16 workers
  const int nw = std::max(1, std::min(workers > 0 ? workers : 16, n));
  std::atomic<int> next{0};
  std::vector<int> rc(n, CB_OK);
  auto work = [&]() {
    (void)hipSetDevice(device);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const int i = order[k];
      out[i] = cb_result{};
      rc[i] = mode[i] == 1 ? cb_solve_force(plans[i], f[i], target[i], p_io[i], nullptr, opts, &out[i])
                           : cb_solve_indent(plans[i], f[i], target[i], p_io[i], nullptr, opts, &out[i]);
      if (out[i].status == CB_OK && rc[i] != CB_OK) out[i].status = rc[i];
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; w++) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  for (int i = 0; i < n; i++)
    if (rc[i] != CB_OK) return cb_fail(rc[i], "problem " + std::to_string(i) + " of the batch failed");
  return CB_OK;
}

// Quasi-static sweeps of independent problems, concurrently (one cb_sweep
// per problem on its plan's stream), the longest (N^2 x steps) first.
extern "C" int cb_sweep_batch(int n, const cb_plan* plans, const double* const* f, const double* const* d_steps,
                              const int* nsteps, double* const* p_state, unsigned char* const* mask_state,
                              const cb_solve_opts* opts, int workers, cb_result* const* out) {
  if (n < 0 || (n > 0 && (!plans || !f || !d_steps || !nsteps || !p_state || !mask_state || !out)))
    return cb_fail(CB_E_INVALID, "null argument or negative count");
  if (n == 0) return CB_OK;
  std::set<const void*> seen;
  for (int i = 0; i < n; i++) {
    if (!plans[i] || !f[i] || !p_state[i] || !mask_state[i] || nsteps[i] < 0 || (nsteps[i] > 0 && (!d_steps[i] || !out[i])))
      return cb_fail(CB_E_INVALID, "null plan, array or result in the batch, or a negative step count");
    if (!seen.insert(plans[i]).second) return cb_fail(CB_E_INVALID, "a plan appears twice in the batch");
  }
  int device = 0;
  CB_HIP(hipGetDevice(&device));
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long long)plans[a]->N * plans[a]->N * nsteps[a] > (long long)plans[b]->N * plans[b]->N * nsteps[b];
  });
  const int nw = std::max(1, std::min(workers > 0 ? workers : 16, n));
  std::atomic<int> next{0};
  std::vector<int> rc(n, CB_OK);
  auto work = [&]() {
    (void)hipSetDevice(device);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const int i = order[k];
      rc[i] = cb_sweep(plans[i], f[i], d_steps[i], nsteps[i], p_state[i], mask_state[i], opts, out[i]);
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; w++) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  for (int i = 0; i < n; i++)
    if (rc[i] != CB_OK) return cb_fail(rc[i], "sweep " + std::to_string(i) + " of the batch failed");
  return CB_OK;
}
