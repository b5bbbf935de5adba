"""Fourier-space fundamental solution of a layer on a half-space (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Eq. 4  (Sec. 2): homogeneous transfer function u_z = 2 p0 / (E* |k|).
  * Eq. 5-8 (Sec. 2): Navier equilibrium, plane-wave ansatz, the two
    second-order ODEs in z, boundary conditions (a)-(d).
  * Eq. 9-10 (Sec. 2): closed-form surface displacement with constants
    A, B, C, D (the constant C is printed over two lines; both lines are
    summed).
  * Eq. 11 (Sec. 2): k = sqrt(kx^2 + ky^2); no value is defined at k = 0.

Reading adopted where the paper is silent:
  * DC term: chosen so that the discrete frequency sum of the transfer
    function equals its integral over the Brillouin zone
    [-pi/Delta, pi/Delta]^2 (see `dc_bz`).  For the homogeneous case this
    makes the self-influence coefficient of a cell equal to the exact one
    of a uniformly loaded square (Love).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.integrate
import scipy.linalg


@dataclass(frozen=True)
class Material:
    """Layer (h, E1, nu1) bonded to a half-space (E2, nu2); Sec. 2, Fig. 1."""

    h: float
    E1: float
    nu1: float
    E2: float
    nu2: float

    @property
    def E1s(self) -> float:
        """Reduced modulus of the coating, E1* = E1 / (1 - nu1^2) (Eq. 4, 12)."""
        return self.E1 / (1.0 - self.nu1 ** 2)

    @property
    def E2s(self) -> float:
        return self.E2 / (1.0 - self.nu2 ** 2)


# ---------------------------------------------------------------------------
# Eq. 9-10 exactly as printed
# ---------------------------------------------------------------------------
def abcd_raw(E1, nu1, E2, nu2):
    """Constants A, B, C, D of Eq. 10 written out term by term."""
    A = (E2 * (3 - 4 * nu1) * (1 + nu1) - E1 * (3 - 4 * nu2) * (1 + nu2)) * (
        E1 * (1 + nu2) - E2 * (1 + nu1))
    B = 4 * (E2 * (1 + nu1) + E1 * (3 - 4 * nu2) * (1 + nu2)) * (
        E1 * (1 + nu2) - E2 * (1 + nu1))
    C = (E1 ** 2 * (4 * nu2 - 3) * (nu2 + 1) ** 2
         - 2 * E1 * E2 * (nu1 + 1) * (2 * nu1 - 1) * (nu2 + 1) * (2 * nu2 - 1)
         + E2 ** 2 * (8 * nu1 ** 2 - 12 * nu1 + 5) * (nu1 + 1) ** 2)
    D = (E2 * (1 + nu1) + E1 * (3 - 4 * nu2) * (1 + nu2)) * (
        E2 * (3 - 4 * nu1) * (1 + nu1) + E1 * (1 + nu2))
    return A, B, C, D


def khat_raw(k, mat: Material):
    """Surface displacement per unit pressure amplitude, Eq. 9 as printed.

    Returns u_z(k)/p0 for k > 0 (array).  Eq. 9 numerator carries
    B*k*h*exp(-2kh), the denominator B*k^2*h^2*exp(-2kh); both are used as
    printed.
    """
    k = np.asarray(k, dtype=np.float64)
    A, B, C, D = abcd_raw(mat.E1, mat.nu1, mat.E2, mat.nu2)
    kh = k * mat.h
    e2 = np.exp(-2.0 * kh)
    e4 = np.exp(-4.0 * kh)
    num = A * e4 + B * kh * e2 + D
    den = -A * e4 - B * kh * kh * e2 + 2.0 * C * e2 + D
    return 2.0 * (1.0 - mat.nu1 ** 2) * num / (k * mat.E1 * den)


# ---------------------------------------------------------------------------
# Normalised form of Eq. 9-10 (same function, no overflow for stiff bases)
# ---------------------------------------------------------------------------
def coeffs_ab(mat: Material):
    """Dimensionless a, b with A/D = -a b, B/D = 4 b, 2C/D = -(a + b).

    Derived from Eq. 10 by dividing every bracket by
    2 (1+nu1)(1+nu2) mu2 with mu_i = E_i / (2 (1+nu_i)),
    alpha = mu1/mu2 and kappa_i = 3 - 4 nu_i:
        a = (alpha kappa2 - kappa1) / (1 + alpha kappa2)
        b = (alpha - 1) / (alpha + kappa1)
    """
    mu1 = mat.E1 / (2.0 * (1.0 + mat.nu1))
    mu2 = mat.E2 / (2.0 * (1.0 + mat.nu2))
    al = mu1 / mu2
    k1 = 3.0 - 4.0 * mat.nu1
    k2 = 3.0 - 4.0 * mat.nu2
    a = (al * k2 - k1) / (1.0 + al * k2)
    b = (al - 1.0) / (al + k1)
    return a, b


def shape_factor(t, mat: Material):
    """C(t) = K^(k) * E1* * k / 2 as a function of t = k h (Eq. 9 / D)."""
    t = np.asarray(t, dtype=np.float64)
    a, b = coeffs_ab(mat)
    e2 = np.exp(-2.0 * t)
    e4 = e2 * e2
    num = 1.0 + 4.0 * b * t * e2 - a * b * e4
    den = 1.0 - (a + b + 4.0 * b * t * t) * e2 + a * b * e4
    return num / den


def khat(k, mat: Material):
    """Transfer function K^(k) = u_z / p0 for k > 0 (Eq. 9, Eq. 11)."""
    k = np.asarray(k, dtype=np.float64)
    return 2.0 / (mat.E1s * k) * shape_factor(k * mat.h, mat)


# ---------------------------------------------------------------------------
# Independent derivation: boundary-value problem of Eq. 5-8 per wavenumber
# ---------------------------------------------------------------------------
def _ode_matrix(k, nu):
    """First-order form y' = M y of Eq. 7-8, y = (u_k, u_z, u_k', u_z')."""
    c1 = 2.0 * (1.0 - nu) * k * k / (1.0 - 2.0 * nu)
    c2 = (1.0 - 2.0 * nu) * k * k / (2.0 * (1.0 - nu))
    M = np.zeros((4, 4), dtype=np.complex128)
    M[0, 2] = 1.0
    M[1, 3] = 1.0
    # Eq. 7: u_k'' = -ik/(1-2nu) u_z' + 2(1-nu)k^2/(1-2nu) u_k
    M[2, 0] = c1
    M[2, 3] = -1j * k / (1.0 - 2.0 * nu)
    # Eq. 8: u_z'' = -ik/(2(1-nu)) u_k' + (1-2nu)k^2/(2(1-nu)) u_z
    M[3, 1] = c2
    M[3, 2] = -1j * k / (2.0 * (1.0 - nu))
    return M


def _stress_rows(k, E, nu):
    """Rows giving (sigma_zz, sigma_kz) from y by Hooke's law."""
    mu = E / (2.0 * (1.0 + nu))
    lam = 2.0 * mu * nu / (1.0 - 2.0 * nu)
    szz = np.array([lam * 1j * k, 0.0, 0.0, lam + 2.0 * mu], dtype=np.complex128)
    skz = np.array([0.0, mu * 1j * k, mu, 0.0], dtype=np.complex128)
    return szz, skz


def bvp_surface_displacement(k, mat: Material, p0=1.0):
    """u_z(z=0) for p = p0 e^{ikr} from Eq. 5-8 with conditions (a)-(d).

    z points into the body; the interface is at z = h.  Unknowns: the layer
    state y(0) (4) and the two amplitudes of the decaying half-space
    solution (2).  Conditions: (b) zero shear and (c) sigma_zz = -p0 at
    z = 0; (a) continuity of u_k, u_z at z = h plus continuity of the
    normal and shear tractions there (a bonded interface; the paper lists
    displacement continuity only); (d) decay with depth, imposed by
    restricting the half-space state to the generalised eigenspace of the
    eigenvalue -k.  Returns the real surface displacement.
    """
    M1 = _ode_matrix(k, mat.nu1)
    M2 = _ode_matrix(k, mat.nu2)
    # decaying solutions e^{-kz}, z e^{-kz}: null space of (M2 + k I)^2
    S = M2 + k * np.eye(4)
    V = scipy.linalg.null_space(S @ S)
    assert V.shape[1] == 2
    szz1, skz1 = _stress_rows(k, mat.E1, mat.nu1)
    szz2, skz2 = _stress_rows(k, mat.E2, mat.nu2)
    Phi = scipy.linalg.expm(M1 * mat.h)  # y_layer(h) = Phi y(0)
    A = np.zeros((6, 6), dtype=np.complex128)
    rhs = np.zeros(6, dtype=np.complex128)
    A[0, :4] = skz1                      # (b)
    A[1, :4] = szz1                      # (c)
    rhs[1] = -p0
    A[2, :4] = Phi[0]                    # (a) u_k
    A[2, 4:] = -V[0]
    A[3, :4] = Phi[1]                    # (a) u_z
    A[3, 4:] = -V[1]
    A[4, :4] = szz1 @ Phi                # traction sigma_zz
    A[4, 4:] = -(szz2 @ V)
    A[5, :4] = skz1 @ Phi                # traction sigma_kz
    A[5, 4:] = -(skz2 @ V)
    sol = np.linalg.solve(A, rhs)
    uz0 = sol[1]
    return uz0.real, abs(uz0.imag)


# ---------------------------------------------------------------------------
# Discrete transfer table on the zero-padded grid, including the DC term
# ---------------------------------------------------------------------------
def grid_wavenumbers(N, L):
    """Wavenumbers of the 2N-padded grid: (ky over M rows, kx over N+1).

    Delta = L/N (Sec. 2, Fig. 2); M = 2N; k = 2 pi fftfreq(M, Delta).
    """
    M = 2 * N
    dx = L / N
    ky = 2.0 * np.pi * np.fft.fftfreq(M, d=dx)
    kx = 2.0 * np.pi * np.fft.rfftfreq(M, d=dx)
    return ky, kx


def brillouin_integral(N, L, mat: Material):
    """Integral of K^ over the Brillouin zone [-pi/D, pi/D]^2 (FP64, quad).

    By the eight-fold symmetry of |k| the square is eight triangles
    0 <= theta <= pi/4, 0 <= k <= (pi/D)/cos(theta); in polar coordinates
    K^(k) k dk dtheta = (2/E1*) C(k h) dk dtheta.
    """
    dx = L / N
    kmax = math.pi / dx

    def inner(theta):
        K = kmax / math.cos(theta)
        f = lambda k: float(shape_factor(k * mat.h, mat))
        pts = None
        if mat.h > 0.0:
            pts = [p for p in (0.5 / mat.h, 2.0 / mat.h, 10.0 / mat.h) if p < K]
        val, _ = scipy.integrate.quad(f, 0.0, K, points=pts, limit=400,
                                      epsabs=0.0, epsrel=1e-13)
        return val

    outer, _ = scipy.integrate.quad(inner, 0.0, math.pi / 4.0, limit=200,
                                    epsabs=0.0, epsrel=1e-13)
    return 8.0 * (2.0 / mat.E1s) * outer


def dc_bz(N, L, mat: Material):
    """DC value making the DFT frequency sum equal the Brillouin integral.

    K^(0) = dk^-2 * Integral_BZ K^ d^2k - sum_{k != 0} K^(k), dk = 2 pi/(M D),
    where the sum runs over all M x M grid wavenumbers except k = 0.
    """
    M = 2 * N
    dx = L / N
    dk = 2.0 * np.pi / (M * dx)
    ky = 2.0 * np.pi * np.fft.fftfreq(M, d=dx)
    kk = np.sqrt(ky[:, None] ** 2 + ky[None, :] ** 2)
    kk[0, 0] = 1.0
    vals = khat(kk, mat)
    vals[0, 0] = 0.0
    return brillouin_integral(N, L, mat) / dk ** 2 - vals.sum()


def transfer_table(N, L, mat: Material, dc_mode="bz"):
    """Real table T[ky, kx] of shape (M, N+1) multiplying rfft2(pad(p)).

    Eq. 11 with k = sqrt(kx^2 + ky^2); the DC entry per `dc_mode`:
    "bz" (Brillouin-zone matched, default) or "zero" (no DC component).
    """
    ky, kx = grid_wavenumbers(N, L)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    kk[0, 0] = 1.0
    T = khat(kk, mat)
    if dc_mode == "bz":
        T[0, 0] = dc_bz(N, L, mat)
    elif dc_mode == "zero":
        T[0, 0] = 0.0
    else:
        raise ValueError(dc_mode)
    return T


def critical_stress(mat: Material, dgamma, dx):
    """sigma_c = sqrt(E1* dgamma / (0.473201 Delta)), Eq. 12."""
    return math.sqrt(mat.E1s * dgamma / (0.473201 * dx))
