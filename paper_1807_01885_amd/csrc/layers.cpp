// Surface compliance K^(k) of a stack of bonded elastic layers on a
// half-space: the layer-on-substrate boundary-value problem of Sec. 2
// (Eq. 5-8, conditions (a)-(d), bonded interfaces as for Eq. 9) written
// for n layers and solved per wavenumber as one real linear system.
//
// With the plane-wave ansatz of Eq. 6, u_k = i U(z), u_z = W(z) (U, W real),
// t = k z and p0 = k, Eq. 7-8 have in every layer the solutions
//   decaying, from the layer top (t >= 0), unknowns (C, d):
//     W = (C + d t) e^-t,           U = ((3 - 4 nu) d - C - d t) e^-t
//   growing, towards the layer bottom (s = t - k h <= 0), unknowns (A, b):
//     W = (A + b s) e^s,            U = (A + (3 - 4 nu) b + b s) e^s
// and the tractions sigma_zz / k = -lambda U + (lambda + 2 mu) W' / k and
// sigma_kz / (i k) = mu (W + U' / k).  No exponential exceeds 1, so the
// system is well conditioned at any k h.  Rows: zero shear and
// sigma_zz = -p0 at the surface; continuity of U, W and both tractions at
// every interface; the half-space keeps its decaying pair.  K^ = W(0) / k.
// (For one layer this is Eq. 9; for none, Eq. 4: W(0) = 2 / (E* k) k.)
#include <cmath>
#include <thread>
#include <vector>

#include "internal.h"

namespace cb {
namespace {

struct Block {
  double lam, mu, kap;  // Lame constants, 3 - 4 nu
};

Block block(double E, double nu) {
  const double mu = E / (2.0 * (1.0 + nu));
  return {2.0 * mu * nu / (1.0 - 2.0 * nu), mu, 3.0 - 4.0 * nu};
}

// Values (U, W, sigma_zz/k, sigma_kz/(ik)) of the two solution pairs of a
// block at local coordinate t (decaying pair) and s (growing pair):
// out[q][c], q the quantity, c the unknown (C, d, A, b).
void decaying(const Block& B, double t, double out[4][2]) {
  const double e = std::exp(-t);
  // per unknown C and d
  const double W[2] = {e, t * e};
  const double U[2] = {-e, (B.kap - t) * e};
  const double Wp[2] = {-e, (1.0 - t) * e};
  const double Up[2] = {e, (t - (B.kap + 1.0)) * e};
  for (int c = 0; c < 2; c++) {
    out[0][c] = U[c];
    out[1][c] = W[c];
    out[2][c] = -B.lam * U[c] + (B.lam + 2.0 * B.mu) * Wp[c];
    out[3][c] = B.mu * (W[c] + Up[c]);
  }
}

void growing(const Block& B, double s, double out[4][2]) {
  const double e = std::exp(s);
  // per unknown A and b
  const double W[2] = {e, s * e};
  const double U[2] = {e, (B.kap + s) * e};
  const double Wp[2] = {e, (1.0 + s) * e};
  const double Up[2] = {e, (B.kap + 1.0 + s) * e};
  for (int c = 0; c < 2; c++) {
    out[0][c] = U[c];
    out[1][c] = W[c];
    out[2][c] = -B.lam * U[c] + (B.lam + 2.0 * B.mu) * Wp[c];
    out[3][c] = B.mu * (W[c] + Up[c]);
  }
}

// Gaussian elimination with partial pivoting on an n x n row-major system;
// returns false if singular.
bool solve_dense(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int c = 0; c < n; c++) {
    int piv = c;
    double best = std::fabs(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; r++) {
      const double v = std::fabs(A[(size_t)r * n + c]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best > 0.0)) return false;
    if (piv != c) {
      for (int j = 0; j < n; j++) std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
      std::swap(b[c], b[piv]);
    }
    const double inv = 1.0 / A[(size_t)c * n + c];
    for (int r = c + 1; r < n; r++) {
      const double f = A[(size_t)r * n + c] * inv;
      if (f == 0.0) continue;
      for (int j = c; j < n; j++) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; r--) {
    double s = b[r];
    for (int j = r + 1; j < n; j++) s -= A[(size_t)r * n + j] * b[j];
    b[r] = s / A[(size_t)r * n + r];
  }
  return true;
}

}  // namespace

double layered_compliance(double k, const LayerStack& S) {
  const int n = (int)S.h.size();
  const int size = 4 * n + 2;
  std::vector<double> A((size_t)size * size, 0.0), rhs(size, 0.0);
  auto col = [&](int blk) { return 4 * blk; };
  auto blockof = [&](int i) { return i < n ? block(S.E[i], S.nu[i]) : block(S.Es, S.nus); };
  // values at the top of block i: (4 quantities) x (its unknowns)
  auto top = [&](int i, double v[4][4]) {
    const Block B = blockof(i);
    double dv[4][2], gv[4][2];
    decaying(B, 0.0, dv);
    if (i < n) growing(B, -k * S.h[i], gv);
    for (int q = 0; q < 4; q++) {
      v[q][0] = dv[q][0];
      v[q][1] = dv[q][1];
      v[q][2] = i < n ? gv[q][0] : 0.0;
      v[q][3] = i < n ? gv[q][1] : 0.0;
    }
  };
  auto bottom = [&](int i, double v[4][4]) {
    const Block B = blockof(i);
    double dv[4][2], gv[4][2];
    decaying(B, k * S.h[i], dv);
    growing(B, 0.0, gv);
    for (int q = 0; q < 4; q++) {
      v[q][0] = dv[q][0];
      v[q][1] = dv[q][1];
      v[q][2] = gv[q][0];
      v[q][3] = gv[q][1];
    }
  };
  auto nunk = [&](int i) { return i < n ? 4 : 2; };
  double v0[4][4];
  top(0, v0);
  for (int c = 0; c < nunk(0); c++) {
    A[(size_t)0 * size + col(0) + c] = v0[3][c];  // no shear
    A[(size_t)1 * size + col(0) + c] = v0[2][c];  // sigma_zz = -p0
  }
  rhs[1] = -1.0;
  int r = 2;
  for (int i = 0; i < n; i++) {
    double vb[4][4], vt[4][4];
    bottom(i, vb);
    top(i + 1, vt);
    for (int q = 0; q < 4; q++, r++) {
      for (int c = 0; c < 4; c++) A[(size_t)r * size + col(i) + c] = vb[q][c];
      for (int c = 0; c < nunk(i + 1); c++) A[(size_t)r * size + col(i + 1) + c] = -vt[q][c];
    }
  }
  if (!solve_dense(A, rhs, size)) return NAN;
  double w0 = 0.0;
  for (int c = 0; c < nunk(0); c++) w0 += v0[1][c] * rhs[col(0) + c];
  return w0 / k;
}

void layered_compliance_grid(const LayerStack& S, double dk, int n, std::vector<double>& out) {
  // out[a][b] = K^(dk sqrt(a^2 + b^2)), a, b in [0, n), out[0][0] left 0;
  // the quadrant is symmetric in (a, b): rows of b <= a, mirrored
  out.assign((size_t)n * n, 0.0);
  unsigned nt = std::thread::hardware_concurrency();
  nt = nt < 1 ? 1 : (nt > 32 ? 32 : nt);
  auto work = [&](unsigned w) {
    for (int a = (int)w; a < n; a += (int)nt)
      for (int b = 0; b <= a; b++) {
        if (a == 0 && b == 0) continue;
        const double v = layered_compliance(dk * std::sqrt((double)a * a + (double)b * b), S);
        out[(size_t)a * n + b] = v;
        out[(size_t)b * n + a] = v;
      }
  };
  std::vector<std::thread> pool;
  for (unsigned w = 1; w < nt; w++) pool.emplace_back(work, w);
  work(0);
  for (auto& t : pool) t.join();
}

}  // namespace cb
