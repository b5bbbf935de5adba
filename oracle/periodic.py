"""The literal periodic operator of Eq. 11 (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passage followed
  * Eq. 11 (Sec. 2): u = IFFT[ K^(k) FFT(p) ] with k = sqrt(kx^2 + ky^2) on
    the N x N grid itself, the surface taken as periodic with period L in
    both directions, and the pressure without a DC component: the k = 0
    term is dropped, so a uniform pressure produces no displacement and u
    has zero mean.  The mean pressure (the load per period) is then
    prescribed, and the mean approach d follows from the solve.

This is the periodic counterpart of `operator.Operator` (which pads to 2N
to reproduce the non-periodic sum of Eq. 1 over the patch).  It has the
same interface, so the solvers of `solvers.py` run on it unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .operator import _WORKERS
from .transfer import Material, khat


def periodic_table(N, L, mat: Material):
    """T[ky, kx] of shape (N, N//2 + 1): K^ at k = 2 pi fftfreq(N, D), T[0,0] = 0."""
    dx = L / N
    ky = 2.0 * np.pi * np.fft.fftfreq(N, d=dx)
    kx = 2.0 * np.pi * np.fft.rfftfreq(N, d=dx)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    kk[0, 0] = 1.0
    T = khat(kk, mat)
    T[0, 0] = 0.0
    return T


class PeriodicOperator:
    """K on the L-periodic N x N grid, Eq. 11 without padding or DC term."""

    def __init__(self, N, L, mat: Material, workers=None):
        self.N = int(N)
        self.M = self.N
        self.L = float(L)
        self.dx = self.L / self.N
        self.mat = mat
        self.T = periodic_table(self.N, self.L, mat)
        self.workers = workers or _WORKERS

    def apply(self, p):
        """u = irfft2(T * rfft2(p)) on the N x N torus."""
        P = scipy.fft.rfft2(np.asarray(p, dtype=np.float64), workers=self.workers)
        return scipy.fft.irfft2(P * self.T, s=(self.N, self.N), workers=self.workers)

    def apply_direct(self, p):
        """The same sum written out: u(x_m) = (1/N^2) sum_k K^(k) e^{i k x_m}
        sum_n p(x_n) e^{-i k x_n} over the N^2 grid wavenumbers (k != 0),
        by explicit complex exponentials.  O(N^4); only for N <= 16."""
        N = self.N
        dx = self.dx
        k1 = 2.0 * np.pi * np.fft.fftfreq(N, d=dx)
        x = np.arange(N) * dx
        E = np.exp(-1j * np.outer(k1, x))                 # E[k, n] = e^{-i k x_n}
        P = E @ np.asarray(p, dtype=np.float64) @ E.T     # P[ky, kx]
        kk = np.sqrt(k1[:, None] ** 2 + k1[None, :] ** 2)
        kk[0, 0] = 1.0
        Kf = khat(kk, self.mat)
        Kf[0, 0] = 0.0
        U = Kf * P
        u = np.conj(E).T @ U @ np.conj(E) / N ** 2
        return u.real

    def dense_matrix(self):
        """K as an explicit N^2 x N^2 matrix (from unit loads; tiny N)."""
        N = self.N
        K = np.empty((N * N, N * N))
        for j in range(N * N):
            e = np.zeros(N * N)
            e[j] = 1.0
            K[:, j] = self.apply(e.reshape(N, N)).ravel()
        return K
