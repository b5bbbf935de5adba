"""Exact influence coefficients of uniformly loaded square cells (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Eq. 1 (Sec. 2, Fig. 2): u = K p over the N x N cells.  Here each cell
    carries a uniform pressure and K[i, j] is the displacement at the centre
    of cell i due to unit pressure over cell j: the non-periodic matrix the
    paper contrasts with the periodic evaluation of Eq. 11 (Sec. 2, the
    discussion after Eq. 11).
  * Eq. 2-3 and Eq. 11 (Sec. 2): a surface load and its displacement are
    related through the 2-D Fourier transform with the transfer function
    K^(k) of Eq. 9-10 (k = |k|), so the displacement due to a load q is the
    inverse transform of K^(k) q^(k).

Definition computed.  For the cell [-a, a]^2 (a = Delta/2) the displacement
at the point x is
    D(x) = (1/4 pi^2) Int K^(|k|) Pi^(k) exp(i k.x) d^2k,
    Pi^(k) = (2 sin(kx a)/kx) (2 sin(ky a)/ky)   (the cell's transform).
With K^(k) = 2/(E* k) + psi(k)/k, E* the reduced modulus of the top layer
and psi(k) = k K^(k) - 2/E* (which decays exponentially at large k: the top
layer hides what lies beneath it at short wavelengths, C -> 1 in Eq. 9):
  * the first term is the homogeneous half-space; its cell integral is
    Love's rectangle formula (closed form, `love_rect`);
  * the second term, in polar coordinates (d^2k = k dk dt cancels 1/k),
        D_R(x, y) = (1/4 pi^2) Int_0^inf psi(k) Int_0^{2 pi}
                    Pi^(k cos t, k sin t) cos(k x cos t) cos(k y sin t) dt dk,
    the inner integral by the trapezoid rule (periodic and analytic in t:
    exponential convergence once the node count exceeds the number of
    oscillations), the outer by composite Gauss-Legendre over [0, k_max]
    with k_max where psi has decayed below double precision.

The DC-FFT table: the (2N)-periodic sequence D_circ[m] = D[|m|] for
|m| < N, D_circ[N] = D[N], whose 2-D DFT T multiplies rfft2(pad(p)) so
that irfft2 gives u_i = sum_j D[|i - j|] p_j on the N x N patch exactly
(the wrapped offsets never reach it).

Pins (tests/test_oracle_exact.py): Love's formula against brute-force
quadrature of the Boussinesq kernel; the Fourier-polar remainder against
the closed rectangle integral of the softened kernel 1/sqrt(r^2 + b^2)
(psi = c exp(-b k)); coated coefficients against a real-space brute force
(Hankel transform by quad, cell integral by dblquad); the homogeneous,
thick- and thin-coating limits; additivity (a K x K block of cells equals
one cell of side K Delta); the FFT apply against the direct O(N^4) sum.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

from .operator import _WORKERS
from .transfer import Material, shape_factor


def love_rect(x, y, a, b, Es):
    """Displacement at (x, y) of a homogeneous half-space (reduced modulus
    Es) under unit pressure on |x'| <= a, |y'| <= b: Love's closed form,
    (1/(pi Es)) sum over the corners of F(X, Y) = X asinh(Y/|X|) +
    Y asinh(X/|Y|) (an antiderivative of 1/sqrt(X^2 + Y^2) in X and Y, up
    to terms in one variable that cancel between corners).  Evaluated in
    extended precision: the corner sum cancels like (a/r)^2 far away."""
    x = np.asarray(x, dtype=np.longdouble)
    y = np.asarray(y, dtype=np.longdouble)
    a = np.longdouble(a)
    b = np.longdouble(b)

    def F(X, Y):
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = np.where(X == 0, 0.0, X * np.arcsinh(Y / np.abs(X)))
            t2 = np.where(Y == 0, 0.0, Y * np.arcsinh(X / np.abs(Y)))
        return t1 + t2

    s = F(x + a, y + b) - F(x + a, y - b) - F(x - a, y + b) + F(x - a, y - b)
    return np.asarray(s / (np.longdouble(math.pi) * np.longdouble(Es)), dtype=np.float64)


def softened_rect(x, y, a, b, beta):
    """Integral of 1/sqrt((x-x')^2 + (y-y')^2 + beta^2) over |x'| <= a,
    |y'| <= b (closed form; the potential of a uniform rectangle at height
    beta): corners of H(X, Y) = X ln(Y + rho) + Y ln(X + rho)
    - beta atan(X Y / (beta rho)), rho = sqrt(X^2 + Y^2 + beta^2)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)

    def H(X, Y):
        rho = np.sqrt(X * X + Y * Y + beta * beta)
        return X * np.log(Y + rho) + Y * np.log(X + rho) - beta * np.arctan(X * Y / (beta * rho))

    return H(x + a, y + b) - H(x + a, y - b) - H(x - a, y + b) + H(x - a, y - b)


def _nodes(kmax, kscale, kfirst, reach, a):
    """Quadrature nodes (kx, ky, weight) of the polar double integral.

    k: composite 16-point Gauss-Legendre on [0, kmax]: panels [0, kfirst],
    then doubling, then uniform, no wider than half a period of the fastest
    cosine (reach = largest |x| + |y| + 2a) nor than kscale (the scale on
    which psi varies; kfirst: that of a feature next to k = 0).  t: midpoint
    trapezoid on [0, 2 pi) with n_t nodes (a multiple of 4), of which the
    first quarter is kept (the integrand is even in kx and in ky) with
    weight 4 (2 pi / n_t).
    """
    width = min(math.pi / reach, kscale)
    edges = [0.0]
    k = kfirst
    while k < width and k < kmax:
        edges.append(k)
        k *= 2.0
    npan = max(1, int(math.ceil((kmax - edges[-1]) / width)))
    edges += list(edges[-1] + (kmax - edges[-1]) * np.arange(1, npan + 1) / npan)
    # about 16 k-nodes per panel times n_t / 4 angles, n_t ~ 1.25 k reach
    est = 16.0 * npan * (0.16 * kmax * reach + 12.0)
    if est > 4e7:
        raise ValueError(f"about {est:.1e} quadrature nodes: offsets too far for this coating's k range")
    g, gw = np.polynomial.legendre.leggauss(16)
    KX, KY, W, KK = [], [], [], []
    for k0, k1 in zip(edges[:-1], edges[1:]):
        ks = 0.5 * (k1 - k0) * g + 0.5 * (k1 + k0)
        ws = 0.5 * (k1 - k0) * gw
        nt = 4 * int(math.ceil((1.25 * k1 * reach + 48.0) / 4.0))
        t = (np.arange(nt // 4) + 0.5) * (2.0 * math.pi / nt)
        KX.append((ks[:, None] * np.cos(t)[None, :]).ravel())
        KY.append((ks[:, None] * np.sin(t)[None, :]).ravel())
        W.append(np.repeat(ws * (4.0 * 2.0 * math.pi / nt), t.size))
        KK.append(np.repeat(ks, t.size))
    kx = np.concatenate(KX)
    ky = np.concatenate(KY)
    w = np.concatenate(W)
    kk = np.concatenate(KK)
    pi_hat = (2.0 * a * np.sinc(kx * a / math.pi)) * (2.0 * a * np.sinc(ky * a / math.pi))
    return kx, ky, w * pi_hat, kk


def remainder_points(xs, ys, a, psi, kmax, kscale, kfirst):
    """D_R at the offsets (xs[i], ys[i]): the polar double integral above,
    one quadrature shared by all points (sized for the farthest)."""
    xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
    ys = np.atleast_1d(np.asarray(ys, dtype=np.float64))
    reach = float(np.max(np.abs(xs) + np.abs(ys))) + 2.0 * a
    kx, ky, wp, kk = _nodes(kmax, kscale, kfirst, reach, a)
    wf = wp * psi(kk)
    out = np.empty(xs.size)
    for i in range(xs.size):
        out[i] = np.sum(wf * np.cos(kx * xs[i]) * np.cos(ky * ys[i]))
    return out / (4.0 * math.pi ** 2)


def remainder_grid(n, dx, psi, kmax, kscale, kfirst, chunk=1 << 16):
    """D_R at the offsets (m dx, q dx), m, q in [0, n]: the same double sum
    as `remainder_points`, whose cos(kx x) cos(ky y) factors separate, taken
    as a matrix product over node chunks."""
    a = 0.5 * dx
    reach = 2.0 * n * dx + 2.0 * a
    kx, ky, wp, kk = _nodes(kmax, kscale, kfirst, reach, a)
    wf = wp * psi(kk)
    pos = np.arange(n + 1) * dx
    out = np.zeros((n + 1, n + 1))
    for s in range(0, kx.size, chunk):
        cx = np.cos(np.outer(pos, kx[s:s + chunk]))
        cy = np.cos(np.outer(pos, ky[s:s + chunk]))
        out += (cx * wf[s:s + chunk]) @ cy.T
    return out / (4.0 * math.pi ** 2)


class Coating:
    """psi(k) = k K^(k) - 2/E1* of one layer on a half-space (Eq. 9).

    k_max: C - 1 ~ t^2 e^{-2t} (t = k h) is below double precision beyond
    t = 24.  kscale: psi varies on the scale 1/h, and for a coating stiffer
    than the substrate on 1/ell, ell = h (E1*/E2*)^{1/3} (the thin stiff
    layer spreads a load over ell; complex poles of C lie about 1/ell from
    the real axis).  kfirst: such a coating also gives C a real pole just
    left of t = 0 (near t = -(E2*/E1*)/2, where the denominator of Eq. 9 is
    nearly zero), so the first panels shrink towards k = 0."""

    def __init__(self, mat: Material):
        self.mat = mat
        self.E1s = mat.E1s
        ratio = mat.E1s / mat.E2s
        self.kmax = 24.0 / mat.h
        self.kscale = 0.25 / (mat.h * max(1.0, ratio) ** (1.0 / 3.0))
        self.kfirst = 0.01 * min(1.0, 1.0 / ratio) / mat.h

    def psi(self, k):
        return (2.0 / self.E1s) * (shape_factor(k * self.mat.h, self.mat) - 1.0)


class Stack:
    """psi(k) of a stack of layers on a half-space (multilayer.py)."""

    def __init__(self, layers, Es, nus):
        from .multilayer import khat_layers, reduced
        self.layers, self.Es, self.nus = layers, Es, nus
        self._khat = khat_layers
        self.E1s = reduced(layers[0][1], layers[0][2])
        H = sum(h for (h, _, _) in layers)
        ratio = max(reduced(E, nu) for (_, E, nu) in layers) / reduced(Es, nus)
        self.kmax = 24.0 / layers[0][0]
        self.kscale = 0.25 / (H * max(1.0, ratio) ** (1.0 / 3.0))
        self.kfirst = 0.01 * min(1.0, 1.0 / ratio) / H

    def psi(self, k):
        return k * self._khat(k, self.layers, self.Es, self.nus) - 2.0 / self.E1s


def influence_points(ms, qs, dx, body):
    """D at the cell offsets (ms[i], qs[i]) (integers) for a Coating or Stack."""
    ms = np.atleast_1d(np.asarray(ms))
    qs = np.atleast_1d(np.asarray(qs))
    x, y = ms * dx, qs * dx
    a = 0.5 * dx
    return love_rect(x, y, a, a, body.E1s) + remainder_points(x, y, a, body.psi, body.kmax, body.kscale,
                                                              body.kfirst)


def influence_grid(N, dx, body):
    """D[m, q] for m, q in [0, N] (offsets in cells) for a Coating or Stack."""
    pos = np.arange(N + 1) * dx
    a = 0.5 * dx
    X, Y = np.meshgrid(pos, pos, indexing="ij")
    return love_rect(X, Y, a, a, body.E1s) + remainder_grid(N, dx, body.psi, body.kmax, body.kscale,
                                                            body.kfirst)


def exact_table(D):
    """T (M, N+1) = rfft2 of the 2N-periodic embedding of D[0..N, 0..N]."""
    N = D.shape[0] - 1
    M = 2 * N
    idx = np.abs(((np.arange(M) + N) % M) - N)  # |m| for m in (-N, N], D_circ[N] = D[N]
    circ = D[np.ix_(idx, idx)]
    return scipy.fft.rfft2(circ, workers=_WORKERS).real


class ExactOperator:
    """K of Eq. 1 with exact cell coefficients, evaluated by DC-FFT (same
    interface as operator.Operator, so the solvers run on it unchanged)."""

    def __init__(self, N, L, mat: Material | None = None, layers=None, Es=None, nus=None, D=None):
        self.N = int(N)
        self.M = 2 * self.N
        self.L = float(L)
        self.dx = self.L / self.N
        self.mat = mat
        if D is None:
            body = Coating(mat) if layers is None else Stack(layers, Es, nus)
            D = influence_grid(self.N, self.dx, body)
        self.D = D
        self.T = exact_table(D)

    def apply(self, p):
        N, M = self.N, self.M
        P = scipy.fft.rfft2(np.asarray(p, dtype=np.float64), s=(M, M), workers=_WORKERS)
        return scipy.fft.irfft2(P * self.T, s=(M, M), workers=_WORKERS)[:N, :N]

    def apply_batch(self, ps):
        N, M = self.N, self.M
        P = scipy.fft.rfft2(np.asarray(ps, dtype=np.float64), s=(M, M), axes=(-2, -1), workers=_WORKERS)
        return scipy.fft.irfft2(P * self.T, s=(M, M), axes=(-2, -1), workers=_WORKERS)[..., :N, :N]

    def apply_direct(self, p):
        """u_i = sum_j D[|i - j|] p_j, the O(N^4) sum of Eq. 1."""
        N = self.N
        u = np.zeros((N, N))
        ar = np.arange(N)
        for i in range(N):
            for j in range(N):
                u[i, j] = np.sum(self.D[np.ix_(np.abs(i - ar), np.abs(j - ar))] * p)
        return u
