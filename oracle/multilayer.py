"""Surface compliance of a stack of bonded layers on a half-space (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Generalises the paper's layer-on-substrate solution (Sec. 2, Eq. 5-9) to n
layers (h_i, E_i, nu_i), i = 1 (top) .. n, bonded to each other and to a
half-space (E_s, nu_s); the paper points to such systems in its
introduction (its reference [5]).  Per wavenumber k the boundary-value
problem of Eq. 5-8 is written out in every layer and solved as one linear
system ("global matrix"):

  * in each layer the plane-wave ansatz of Eq. 6 turns Eq. 7-8 into
    y' = M y, y = (u_k, u_z, u_k', u_z'); with t = k z and the scaled state
    (u_k, u_z, u_k'/k, u_z'/k) the matrix is k M~(nu), M~ independent of k;
  * M~ has the double eigenvalues -1 and +1.  A layer's solution is a
    combination of the decaying generalised eigenvectors, referenced to its
    top (e^{-t} (I + (M~ + I) t) v), and of the growing ones, referenced to
    its bottom (e^{s} (I + (M~ - I) s) w, s = t - k h_i <= 0): no exponential
    exceeds 1, so the system stays well conditioned at any k h;
  * the half-space keeps the decaying pair only (condition (d));
  * rows: zero shear and sigma_zz = -p0 at z = 0 (conditions (b), (c));
    at every interface continuity of u_k, u_z (condition (a)) and of
    sigma_zz, sigma_kz (a bonded interface, as read for Eq. 9).

The generalised eigenvectors are null spaces computed numerically from
M~, so the construction carries no closed-form ansatz of its own.
"""
from __future__ import annotations

import functools
import math

import numpy as np
import scipy.integrate
import scipy.linalg

from .transfer import _ode_matrix, _stress_rows


def _scaled_matrix(nu):
    """M~ with M(k) = k D M~ D^-1, D = diag(1, 1, k, k) (state scaled by k)."""
    M = _ode_matrix(1.0, nu)
    return M


@functools.lru_cache(maxsize=64)
def _pairs(nu):
    Mt = _scaled_matrix(nu)
    I = np.eye(4)
    V = scipy.linalg.null_space((Mt + I) @ (Mt + I))   # decaying e^{-t}
    W = scipy.linalg.null_space((Mt - I) @ (Mt - I))   # growing e^{+t}
    assert V.shape[1] == 2 and W.shape[1] == 2
    return Mt, V, W


def _stress_scaled(E, nu):
    """(sigma_zz, sigma_kz) / k as rows acting on the scaled state."""
    return _stress_rows(1.0, E, nu)


def _state_dec(Mt, V, t):
    """Scaled states of the decaying pair at local t >= 0 (array): (..., 4, 2)."""
    t = np.asarray(t, dtype=np.float64)[..., None, None]
    return np.exp(-t) * (np.eye(4) + (Mt + np.eye(4)) * t) @ V


def _state_gro(Mt, W, s):
    """Scaled states of the growing pair at s = t - k h <= 0 (array): (..., 4, 2)."""
    s = np.asarray(s, dtype=np.float64)[..., None, None]
    return np.exp(s) * (np.eye(4) + (Mt - np.eye(4)) * s) @ W


def surface_compliance(k, layers, Es, nus):
    """u_z(0) / p0 for p = p0 e^{ikr}, k > 0 (scalar or array).

    layers: sequence of (h, E, nu) from the top; Es, nus: the half-space.
    """
    k = np.asarray(k, dtype=np.float64)
    shape = k.shape
    k = k.ravel()
    K = k.size
    n = len(layers)
    blocks = [(_pairs(float(nu)), E, nu, h) for (h, E, nu) in layers] + [(_pairs(float(nus)), Es, nus, None)]
    size = 4 * n + 2
    A = np.zeros((K, size, size), dtype=np.complex128)
    rhs = np.zeros((K, size), dtype=np.complex128)
    zero = np.zeros(K)

    def top_states(i):
        """Scaled states (K, 4, unknowns) at the top of block i."""
        (Mt, V, W), _, _, h = blocks[i]
        if h is None:
            return _state_dec(Mt, V, zero)
        return np.concatenate([_state_dec(Mt, V, zero), _state_gro(Mt, W, -k * h)], axis=-1)

    def bottom_states(i):
        (Mt, V, W), _, _, h = blocks[i]
        return np.concatenate([_state_dec(Mt, V, k * h), _state_gro(Mt, W, zero)], axis=-1)

    def stress(i):
        _, E, nu, _ = blocks[i]
        return _stress_rows(1.0, E, nu)

    def cols(i):
        return slice(4 * i, 4 * i + 4) if i < n else slice(4 * n, 4 * n + 2)

    Y0 = top_states(0)
    szz, skz = stress(0)
    A[:, 0, cols(0)] = np.einsum("q,kqc->kc", skz, Y0)    # (b) no shear
    A[:, 1, cols(0)] = np.einsum("q,kqc->kc", szz, Y0)    # (c) sigma_zz = -p0 (p0 = k: scaled)
    rhs[:, 1] = -1.0
    r = 2
    for i in range(n):
        Yb = bottom_states(i)
        Yt = top_states(i + 1)
        sb = stress(i)
        st = stress(i + 1)
        for q in (0, 1):                                   # (a) u_k, u_z
            A[:, r, cols(i)] = Yb[:, q]
            A[:, r, cols(i + 1)] = -Yt[:, q]
            r += 1
        for rb, rt in ((sb[0], st[0]), (sb[1], st[1])):   # sigma_zz, sigma_kz
            A[:, r, cols(i)] = np.einsum("q,kqc->kc", rb, Yb)
            A[:, r, cols(i + 1)] = -np.einsum("q,kqc->kc", rt, Yt)
            r += 1
    x = np.linalg.solve(A, rhs[..., None])[..., 0]
    uz0 = np.einsum("kc,kc->k", Y0[:, 1, :], x[:, cols(0)])
    # scaled load p0 = k: the compliance is u_z / k
    out = uz0.real / k
    return out.reshape(shape) if shape else float(out[0])


def khat_layers(k, layers, Es, nus):
    """K^(k) for an array of k > 0 (Eq. 11 with the multi-layer compliance)."""
    k = np.asarray(k, dtype=np.float64)
    uniq, inv = np.unique(k.ravel(), return_inverse=True)
    vals = np.concatenate([surface_compliance(uniq[i:i + 65536], layers, Es, nus)
                           for i in range(0, uniq.size, 65536)])
    return vals[inv].reshape(k.shape)


def reduced(E, nu):
    return E / (1.0 - nu * nu)


def brillouin_integral_layers(N, L, layers, Es, nus):
    """Integral of K^ over [-pi/D, pi/D]^2 for the stack (quad, polar form)."""
    dx = L / N
    kmax = math.pi / dx
    E1s = reduced(layers[0][1], layers[0][2]) if layers else reduced(Es, nus)
    hs = [h for (h, _, _) in layers] or [1.0]
    H = sum(hs)

    def inner(theta):
        K = kmax / math.cos(theta)
        def f(q):
            q = q if q > 0 else 1e-12 / H
            return surface_compliance(q, layers, Es, nus) * q * E1s / 2.0
        pts = sorted({p for h in hs + [H] for p in (0.5 / h, 2.0 / h, 10.0 / h) if p < K})
        val, _ = scipy.integrate.quad(f, 0.0, K, points=pts or None, limit=400, epsabs=0.0, epsrel=1e-12)
        return val

    outer, _ = scipy.integrate.quad(inner, 0.0, math.pi / 4.0, limit=200, epsabs=0.0, epsrel=1e-12)
    return 8.0 * (2.0 / E1s) * outer


def transfer_table_layers(N, L, layers, Es, nus):
    """Real table (M, N+1) for the 2N-padded operator, DC Brillouin-matched."""
    M = 2 * N
    dx = L / N
    ky = 2.0 * np.pi * np.fft.fftfreq(M, d=dx)
    kx = 2.0 * np.pi * np.fft.rfftfreq(M, d=dx)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    kk[0, 0] = 1.0
    T = khat_layers(kk, layers, Es, nus)
    full = np.sqrt(ky[:, None] ** 2 + ky[None, :] ** 2)
    full[0, 0] = 1.0
    vals = khat_layers(full, layers, Es, nus)
    vals[0, 0] = 0.0
    dk = 2.0 * np.pi / (M * dx)
    T[0, 0] = brillouin_integral_layers(N, L, layers, Es, nus) / dk ** 2 - vals.sum()
    return T


def periodic_table_layers(N, L, layers, Es, nus):
    """(N, N//2+1) table of the L-periodic operator of the stack, no DC term."""
    dx = L / N
    ky = 2.0 * np.pi * np.fft.fftfreq(N, d=dx)
    kx = 2.0 * np.pi * np.fft.rfftfreq(N, d=dx)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    kk[0, 0] = 1.0
    T = khat_layers(kk, layers, Es, nus)
    T[0, 0] = 0.0
    return T


class LayeredOperator:
    """u = K p for a stack on the 2N-padded grid (as operator.Operator), or
    on the L-periodic grid without DC (as periodic.PeriodicOperator)."""

    def __init__(self, N, L, layers, Es, nus, periodic=False):
        from .operator import _WORKERS
        self.N = int(N)
        self.M = self.N if periodic else 2 * self.N
        self.L = float(L)
        self.dx = self.L / self.N
        self.periodic = periodic
        self.T = (periodic_table_layers if periodic else transfer_table_layers)(self.N, self.L, list(layers),
                                                                                Es, nus)
        self.workers = _WORKERS

    def apply(self, p):
        import scipy.fft
        M, N = self.M, self.N
        P = scipy.fft.rfft2(np.asarray(p, dtype=np.float64), s=(M, M), workers=self.workers)
        return scipy.fft.irfft2(P * self.T, s=(M, M), workers=self.workers)[:N, :N]
