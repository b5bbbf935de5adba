"""The discrete surface operator u = K p (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Eq. 1 (Sec. 2): u = K p on the N x N grid of cells of size Delta = L/N
    (Fig. 2), K of size N^2 x N^2.
  * Eq. 2 and Eq. 11 (Sec. 2): K p evaluated as IFFT[ K^ . FFT(p) ].

Reading adopted: the pressure grid is zero-padded to
M = 2N in both directions so that the periodic convolution of Eq. 11
equals the non-periodic sum of Eq. 1 over the N x N patch; forward FFT
unnormalised, inverse 1/M^2 (numpy conventions).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from .transfer import Material, transfer_table

_WORKERS = os.cpu_count() or 1


class Operator:
    """K for one grid (N, L) and one material; the table is built once."""

    def __init__(self, N, L, mat: Material, dc_mode="bz", workers=None):
        self.N = int(N)
        self.M = 2 * self.N
        self.L = float(L)
        self.dx = self.L / self.N
        self.mat = mat
        self.T = transfer_table(self.N, self.L, mat, dc_mode)
        self.workers = workers or _WORKERS

    def apply(self, p):
        """u = irfft2(T * rfft2(pad(p)))[:N, :N]  (Eq. 11 on the padded grid)."""
        N, M = self.N, self.M
        P = scipy.fft.rfft2(np.asarray(p, dtype=np.float64), s=(M, M),
                            workers=self.workers)
        u = scipy.fft.irfft2(P * self.T, s=(M, M), workers=self.workers)
        return u[:N, :N]

    def apply_batch(self, ps):
        """Apply to a stack of fields (B, N, N)."""
        N, M = self.N, self.M
        P = scipy.fft.rfft2(np.asarray(ps, dtype=np.float64), s=(M, M),
                            axes=(-2, -1), workers=self.workers)
        u = scipy.fft.irfft2(P * self.T, s=(M, M), axes=(-2, -1),
                             workers=self.workers)
        return u[..., :N, :N]

    # ---- direct forms, for tiny grids only ---------------------------------
    def kernel_direct(self):
        """Real-space kernel G[m, n] on the M x M torus by explicit DFT sums.

        G[m, n] = (1/M^2) sum_{ky, kx} K^(ky, kx) exp(i (ky m + kx n) Delta),
        the full (not half) spectrum rebuilt from the table by its evenness
        in kx.  O(M^4); only for M <= 64.
        """
        N, M = self.N, self.M
        full = np.empty((M, M))
        full[:, : N + 1] = self.T
        full[:, N + 1:] = self.T[:, 1:N][:, ::-1]
        idx = np.arange(M)
        # exp(2 pi i a b / M): the grid wavenumber times the grid position
        E = np.exp(2j * np.pi * np.outer(idx, idx) / M)
        G = np.einsum("am,ab,bn->mn", E, full, E) / M ** 2
        return G.real, np.abs(G.imag).max()

    def apply_direct(self, p):
        """u_i = sum_j G[(i - j) mod M] p_j, the O(N^4) sum of Eq. 1."""
        G, _ = self.kernel_direct()
        N, M = self.N, self.M
        u = np.zeros((N, N))
        for i in range(N):
            for j in range(N):
                di = (i - np.arange(N)) % M
                dj = (j - np.arange(N)) % M
                u[i, j] = np.sum(G[np.ix_(di, dj)] * p)
        return u

    def dense_matrix(self):
        """K as an explicit N^2 x N^2 matrix (row-major cell order), Eq. 1.

        Built from the FFT kernel (the apply of a unit pressure at cell 0
        gives the kernel over all offsets), so it is only as independent
        as `apply`; `apply_direct` is the independent check.
        """
        N, M = self.N, self.M
        e = np.zeros((N, N))
        e[0, 0] = 1.0
        P = scipy.fft.rfft2(e, s=(M, M))
        g = scipy.fft.irfft2(P * self.T, s=(M, M))  # g[m, n] = G[m, n]
        ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        ii = ii.ravel()
        jj = jj.ravel()
        di = (ii[:, None] - ii[None, :]) % M
        dj = (jj[:, None] - jj[None, :]) % M
        return g[di, dj]
