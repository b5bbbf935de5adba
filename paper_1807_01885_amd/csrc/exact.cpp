// Exact influence coefficients of uniformly loaded square cells and the
// DC-FFT table built from them (kernel mode CB_KERNEL_EXACT).
//
// Eq. 1 with piecewise-constant pressure: K[i][j] is the displacement at the
// centre of cell i due to unit pressure over cell j, the cell integral of the
// point-load Green's function
//   G(r) = (1/2 pi) int_0^inf K^(k) J0(k r) k dk,
// the inverse 2-D Fourier transform of the radial K^ (Eq. 2-3 and 11).  With
// s(k) = k K^(k), which tends to 2/E1* at large k (C -> 1 in Eq. 9; E1* the
// top layer's reduced modulus) and to 2/Es* at k = 0 (the substrate), let
// psi0 = 2/Es* - 2/E1* and b the total coating thickness:
//   G(r) = 1 / (pi E1* r)                       homogeneous top layer
//        + psi0 / (2 pi sqrt(r^2 + b^2))         substrate far field, softened
//        + g(r),  g(r) = (1/2 pi) int_0^inf q(k) J0(k r) dk,
//                 q(k) = s(k) - 2/E1* - psi0 e^{-b k}.
// q vanishes at k = 0 and decays like e^{-2 k h_top}, so g is smooth and
// bounded and falls off like r^-3.
//  * Cells within Chebyshev distance kNear of the point: the first two parts
//    by their closed rectangle integrals (Love's formula; the potential of a
//    uniform rectangle at height b), g by the polar form
//    int dtheta [G1(R_out) - G1(R_in)] over the rays crossing the cell, with
//    G1(R) = int_0^R g(r) r dr = (1/2 pi) int q(k) R J1(k R) / k dk.
//  * Farther cells: tensor Gauss-Legendre over the cell of the whole G, its
//    order set by the distance (the 1/r singularity's Bernstein ellipse).
// g and G1 are piecewise Chebyshev interpolants in r whose nodes are Hankel
// integrals by composite Gauss-Legendre rules in k (one per radial panel):
// panels no wider than half a period of J0 at the panel's largest r nor
// than the scale on which q varies
// (1/ell: a coating much stiffer than the substrate spreads load over
// ell = H (E1*/Es*)^{1/3}, and the poles of C nearest k = 0 lie about 1/ell
// away), up to k where q has decayed below double precision.
//
// The table is the 2-D DFT of the (2N)-periodic embedding D_circ[m] = D[|m|]
// (|m| < N), D_circ[N] = D[N]: a DCT-I of D in each direction, by a radix-2
// complex FFT of length 2N per line.  The padded convolution with it is the
// exact non-periodic sum of Eq. 1 over the patch (wrapped offsets never
// reach it).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "internal.h"

namespace cb {
namespace {

constexpr int kNear = 2;  // Chebyshev radius (in cells) of the polar near field

template <class F>
void parallel_for(int n, F f) {
  unsigned nt = std::thread::hardware_concurrency();
  nt = nt < 1 ? 1 : (nt > 16 ? 16 : nt);
  if ((int)nt > n) nt = n < 1 ? 1 : (unsigned)n;
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) break;
      f(i);
    }
  };
  std::vector<std::thread> pool;
  for (unsigned w = 1; w < nt; w++) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
}

// Piecewise Chebyshev interpolant on panels [edge[p], edge[p+1]].
struct Cheb {
  std::vector<double> edge;
  int n = 0;
  std::vector<double> c;  // n coefficients per panel
  int panels() const { return (int)edge.size() - 1; }
  double node(int p, int j) const {
    const double mid = 0.5 * (edge[p] + edge[p + 1]), half = 0.5 * (edge[p + 1] - edge[p]);
    return mid + half * std::cos(M_PI * (j + 0.5) / n);
  }
  void fit(const std::vector<double>& vals) {  // vals panel-major at node(p, j)
    c.assign(vals.size(), 0.0);
    for (int p = 0; p < panels(); p++)
      for (int k = 0; k < n; k++) {
        double s = 0.0;
        for (int j = 0; j < n; j++) s += vals[(size_t)p * n + j] * std::cos(M_PI * k * (j + 0.5) / n);
        c[(size_t)p * n + k] = (k == 0 ? 1.0 : 2.0) * s / n;
      }
  }
  double operator()(double r) const {
    int p = (int)(std::upper_bound(edge.begin(), edge.end(), r) - edge.begin()) - 1;
    p = p < 0 ? 0 : (p >= panels() ? panels() - 1 : p);
    const double mid = 0.5 * (edge[p] + edge[p + 1]), half = 0.5 * (edge[p + 1] - edge[p]);
    const double x = (r - mid) / half;
    const double* cc = c.data() + (size_t)p * n;
    double b1 = 0.0, b2 = 0.0;
    for (int k = n - 1; k >= 1; k--) {
      const double b0 = 2.0 * x * b1 - b2 + cc[k];
      b2 = b1;
      b1 = b0;
    }
    return x * b1 - b2 + cc[0];
  }
};

// Love's rectangle formula without the 1/(pi E*) factor: the integral of
// 1/sqrt((x-x')^2 + (y-y')^2) over |x'|, |y'| <= a, by the corners of
// F(X, Y) = X asinh(Y/|X|) + Y asinh(X/|Y|).
double love_sq(double x, double y, double a) {
  auto F = [](double X, double Y) {
    const double t1 = X == 0.0 ? 0.0 : X * std::asinh(Y / std::fabs(X));
    const double t2 = Y == 0.0 ? 0.0 : Y * std::asinh(X / std::fabs(Y));
    return t1 + t2;
  };
  return F(x + a, y + a) - F(x + a, y - a) - F(x - a, y + a) + F(x - a, y - a);
}

// Integral of 1/sqrt((x-x')^2 + (y-y')^2 + b^2) over |x'|, |y'| <= a: corners
// of X asinh(Y / sqrt(X^2 + b^2)) + Y asinh(X / sqrt(Y^2 + b^2))
// - b atan(X Y / (b rho)), rho = sqrt(X^2 + Y^2 + b^2).
double soft_sq(double x, double y, double a, double b) {
  auto H = [b](double X, double Y) {
    const double rho = std::sqrt(X * X + Y * Y + b * b);
    return X * std::asinh(Y / std::sqrt(X * X + b * b)) + Y * std::asinh(X / std::sqrt(Y * Y + b * b)) -
           b * std::atan(X * Y / (b * rho));
  };
  return H(x + a, y + a) - H(x + a, y - a) - H(x - a, y + a) + H(x - a, y - a);
}

// In-place radix-2 complex DFT, X[k] = sum_j x[j] exp(-2 pi i j k / M).
void fft_radix2(std::vector<std::complex<double>>& x, const std::vector<std::complex<double>>& tw) {
  const int M = (int)x.size();
  for (int i = 1, j = 0; i < M; i++) {
    int bit = M >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  for (int len = 2; len <= M; len <<= 1) {
    const int half = len >> 1, step = M / len;
    for (int i = 0; i < M; i += len)
      for (int j = 0; j < half; j++) {
        const std::complex<double> u = x[i + j], v = x[i + j + half] * tw[(size_t)j * step];
        x[i + j] = u + v;
        x[i + j + half] = u - v;
      }
  }
}

}  // namespace

int exact_influence(int N, double L, const LayerStack& S, std::vector<double>& D, std::vector<double>& T) {
  const int NC = N + 1;
  const double dx = L / N, a = 0.5 * dx;
  const double Et = S.h.empty() ? S.Es / (1.0 - S.nus * S.nus) : S.E[0] / (1.0 - S.nu[0] * S.nu[0]);
  const double Esub = S.Es / (1.0 - S.nus * S.nus);
  double H = 0.0;
  for (double x : S.h) H += x;
  const double htop = S.h.empty() ? 0.0 : S.h[0];
  const double psi0 = 2.0 / Esub - 2.0 / Et;
  // a stack of layers all of the substrate's material is a half-space
  bool coated = false;
  double emax = 0.0;
  for (size_t i = 0; i < S.h.size(); i++) {
    if (S.E[i] != S.Es || S.nu[i] != S.nus) coated = true;
    emax = std::max(emax, S.E[i] / (1.0 - S.nu[i] * S.nu[i]));
  }
  // softening length: e^{-b k} must decay at least as fast as q (e^{-2 k h})
  const double b = 2.0 * H;
  // length over which a coating stiffer than the substrate spreads a load:
  // the poles of C nearest k = 0 lie about 1/ell from the real axis
  const double ell = H * std::cbrt(std::max(1.0, emax / Esub));
  if (coated && htop < dx / 8.0)
    return cb_fail(CB_E_UNSUPPORTED, "the exact kernel needs a top layer at least Delta/8 thick (h = " +
                                         std::to_string(htop) + ", Delta = " + std::to_string(dx) + ")");
  const Coef cf = S.h.size() == 1 ? coefficients(S.E[0], S.nu[0], S.Es, S.nus) : Coef{0.0, 0.0};

  // ---- radial tables of g (far field) and G1 (near field) ------------------
  Cheb gt, g1;
  const double rmax = std::sqrt(2.0) * (N + 0.5) * dx * (1.0 + 1e-9);
  if (coated) {
    {
      double r = (kNear + 0.5) * dx * (1.0 - 1e-9);
      gt.edge.push_back(r);
      // panels no wider than h_top while terms decaying like e^{-r/h_top}
      // matter, then 2 ell while those on the scale ell do, then doubling
      while (r < rmax) {
        const double next = r < 40.0 * htop ? std::min(r + htop, 40.0 * htop)
                            : r < 40.0 * ell ? std::min(r + 2.0 * ell, 40.0 * ell)
                                             : 2.0 * r;
        r = next > r ? next : 2.0 * r;
        gt.edge.push_back(std::min(r, rmax));
      }
      gt.n = 24;
    }
    {
      const double r0 = 0.5 * dx * (1.0 - 1e-9), r1 = (kNear + 0.5) * std::sqrt(2.0) * dx * (1.0 + 1e-9);
      const double w = std::min(2.0 * htop, 0.5 * dx);
      const int np = (int)std::ceil((r1 - r0) / w);
      for (int p = 0; p <= np; p++) g1.edge.push_back(r0 + (r1 - r0) * p / np);
      g1.n = 24;
    }
    // k rules, one per radial panel: edges doubling from k0 towards the
    // uniform width, then uniform, the width no more than half a period of
    // J0 at the panel's outer radius nor than 1/(4 ell).  For a coating
    // stiffer than the substrate C has a real pole just left of k = 0, near
    // t = -(Es*/E1*)/2: the first panels stay well inside the distance to it
    std::vector<double> gx, gw;
    gauss_legendre(12, gx, gw);
    const double kmax = 24.0 / htop;
    struct Rule {
      std::vector<double> k, w;  // nodes, weights times q(k) / (2 pi)
    };
    auto make_rule = [&](double rcap, Rule& R) {
      const double width = std::min(M_PI / rcap, 0.25 / ell);
      std::vector<double> ke{0.0};
      double k = 0.01 * std::min(1.0, Esub / emax) / H;
      while (k < width && k < kmax) {
        ke.push_back(k);
        k *= 2.0;
      }
      const double k1 = ke.back();
      const long long nu = (long long)std::ceil((kmax - k1) / width);
      for (long long p = 1; p <= nu; p++) ke.push_back(k1 + (kmax - k1) * (double)p / (double)nu);
      const size_t nk = (ke.size() - 1) * 12;
      R.k.resize(nk);
      R.w.resize(nk);
      for (size_t p = 0; p + 1 < ke.size(); p++) {
        const double mid = 0.5 * (ke[p] + ke[p + 1]), half = 0.5 * (ke[p + 1] - ke[p]);
        for (int i = 0; i < 12; i++) {
          const double kq = mid + half * gx[i];
          double s;
          if (S.h.size() == 1) {
            const double t = kq * htop, e2 = std::exp(-2.0 * t), e4 = e2 * e2;
            const double den = 1.0 - (cf.a + cf.b + 4.0 * cf.b * t * t) * e2 + cf.a * cf.b * e4;
            const double num = (cf.a + cf.b + 4.0 * cf.b * t + 4.0 * cf.b * t * t) * e2 - 2.0 * cf.a * cf.b * e4;
            s = (2.0 / Et) * (num / den);  // (2/E1*) (C - 1)
          } else {
            s = kq * layered_compliance(kq, S) - 2.0 / Et;
          }
          R.k[p * 12 + i] = kq;
          R.w[p * 12 + i] = half * gw[i] * (s - psi0 * std::exp(-b * kq)) / (2.0 * M_PI);
        }
      }
    };
    const int pg = gt.panels(), p1 = g1.panels();
    std::vector<Rule> rules(pg + p1);
    parallel_for(pg + p1, [&](int p) { make_rule(p < pg ? gt.edge[p + 1] : g1.edge[p - pg + 1], rules[p]); });
    const int ng = pg * gt.n, n1 = p1 * g1.n;
    std::vector<double> gv(ng), g1v(n1);
    parallel_for(ng + n1, [&](int i) {
      double s = 0.0;
      if (i < ng) {
        const Rule& R = rules[i / gt.n];
        const double r = gt.node(i / gt.n, i % gt.n);
        for (size_t j = 0; j < R.k.size(); j++) s += R.w[j] * ::j0(R.k[j] * r);
        gv[i] = s;
      } else {
        const int q = i - ng;
        const Rule& R = rules[pg + q / g1.n];
        const double Rr = g1.node(q / g1.n, q % g1.n);
        for (size_t j = 0; j < R.k.size(); j++) s += R.w[j] * ::j1(R.k[j] * Rr) / R.k[j];
        g1v[q] = s * Rr;
      }
    });
    gt.fit(gv);
    g1.fit(g1v);
  }

  // ---- coefficients ----------------------------------------------------------
  D.assign((size_t)NC * NC, 0.0);
  std::vector<std::vector<double>> glx(13), glw(13);
  for (int n = 4; n <= 12; n++) gauss_legendre(n, glx[n], glw[n]);
  std::vector<double> px, pw;
  gauss_legendre(32, px, pw);
  const double cG = 1.0 / (M_PI * Et), cS = psi0 / (2.0 * M_PI);
  auto Gfull = [&](double r) {
    double v = cG / r;
    if (coated) v += cS / std::sqrt(r * r + b * b) + gt(r);
    return v;
  };
  // polar integral of G1 over the rays from the origin through cell (m, q)
  auto polar = [&](int m, int q) {
    if (m == 0 && q == 0) {
      double s = 0.0;
      for (int i = 0; i < 32; i++) {
        const double th = (M_PI / 8.0) * (1.0 + px[i]);
        s += pw[i] * g1(a / std::cos(th));
      }
      return 8.0 * (M_PI / 8.0) * s;
    }
    const double xl = (m - 0.5) * dx, xh = (m + 0.5) * dx, yl = (q - 0.5) * dx, yh = (q + 0.5) * dx;
    double th[4] = {std::atan2(yl, xl), std::atan2(yh, xl), std::atan2(yl, xh), std::atan2(yh, xh)};
    std::sort(th, th + 4);
    double s = 0.0;
    for (int seg = 0; seg < 3; seg++) {
      const double t0 = th[seg], t1 = th[seg + 1];
      if (!(t1 > t0)) continue;
      double ss = 0.0;
      for (int i = 0; i < 32; i++) {
        const double t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * px[i];
        const double c = std::cos(t), sn = std::sin(t);
        double lo = xl / c, hi = xh / c;  // c > 0: the cell lies at x > 0
        if (sn > 0.0) {
          lo = std::max(lo, yl / sn);
          hi = std::min(hi, yh / sn);
        } else if (sn < 0.0) {
          lo = std::max(lo, yh / sn);
          hi = std::min(hi, yl / sn);
        }
        if (hi > lo) ss += pw[i] * (g1(hi) - g1(lo));
      }
      s += 0.5 * (t1 - t0) * ss;
    }
    return s;
  };
  parallel_for(NC, [&](int m) {
    for (int q = 0; q <= m; q++) {
      const double x = m * dx, y = q * dx;
      double v;
      if (m <= kNear) {
        v = cG * love_sq(x, y, a);
        if (coated) v += cS * soft_sq(x, y, a, b) + polar(m, q);
      } else {
        const double rho = 2.0 * m + std::sqrt(4.0 * m * m - 1.0);
        int n = (int)std::ceil(19.6 / std::log(rho)) + 1;
        n = n < 4 ? 4 : (n > 12 ? 12 : n);
        if (coated && htop < dx && std::hypot(x, y) < 40.0 * htop) n = 12;
        const std::vector<double>& gxn = glx[n];
        const std::vector<double>& gwn = glw[n];
        double s = 0.0;
        for (int i = 0; i < n; i++) {
          const double xi = x + a * gxn[i];
          double si = 0.0;
          for (int j = 0; j < n; j++) si += gwn[j] * Gfull(std::hypot(xi, y + a * gxn[j]));
          s += gwn[i] * si;
        }
        v = a * a * s;
      }
      D[(size_t)m * NC + q] = v;
      D[(size_t)q * NC + m] = v;
    }
  });

  // ---- DCT-I in both directions: T = DFT of the 2N-periodic embedding -------
  const int M = 2 * N;
  std::vector<std::complex<double>> tw(M / 2);
  for (int j = 0; j < M / 2; j++) tw[j] = std::polar(1.0, -2.0 * M_PI * j / M);
  std::vector<double> R((size_t)NC * NC);
  auto dct_lines = [&](const std::vector<double>& in, std::vector<double>& out) {
    // out[a][line] = sum_j in[line][|j|] e^{-2 pi i a j / M}: transforms the
    // second index of `in`, written transposed so that two passes give T
    parallel_for(NC, [&](int line) {
      std::vector<std::complex<double>> x(M);
      const double* src = in.data() + (size_t)line * NC;
      for (int j = 0; j <= N; j++) x[j] = src[j];
      for (int j = 1; j < N; j++) x[M - j] = src[j];
      fft_radix2(x, tw);
      for (int k = 0; k <= N; k++) out[(size_t)k * NC + line] = x[k].real();
    });
  };
  dct_lines(D, R);
  T.assign((size_t)NC * NC, 0.0);
  dct_lines(R, T);
  return CB_OK;
}

}  // namespace cb
