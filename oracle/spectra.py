"""Spectra on the periodic FFT mesh.

* Wavenumber ordering, eq. (Kvalues) of Appendix B: k_d = 2 pi j / (N h) for
  j <= N/2, else -2 pi (N - j) / (N h).  The grid spacing h is taken as the
  period over N (a periodic grid); the appendix's L/(N-1) is a vertex-grid
  convention that does not describe a periodic FFT mesh.
* Analytic weight-function transforms, Appendix B, eqs. (OmegaHat2),
  (omegaHat0and1), (omegaHat3), (omegaHatV2) and their k -> 0 limits.  They are
  written through the spherical Bessel functions j0, j1 (scipy), which evaluate
  the printed closed forms without cancellation at small kR.
* Vector-weight convention on the Nyquist plane: with j_d = N_d/2 taken on the
  positive side, component d of the vector spectrum is not Hermitian there; the
  oracle sets that component to zero on that plane (the mean of its values at
  +pi/h and -pi/h), which keeps every convolution exactly real and makes the
  back-convolution the exact transpose of the forward one.
* Bulk-fluid kernel transform, eq. (CplusPsiHat) with the ball moments I_{-1},
  I_0, I_1 of the bulk-fluid section and their k -> 0 limits.  The prefactor is
  the one that the real-space kernel eq. (CplusPsiFunc) transforms to,
  (z_i z_j l_B / 2) (4 pi / k): the printed transform carries twice that value.
  For kR < 1 the closed forms are evaluated with 40-digit mpmath arithmetic.
* Poisson denominators: eigenvalues of the 7-point finite-difference Laplacian,
  sum_d 2 (1 - cos(k_d h_d)) / h_d^2 (eq. (potentialSolution), read with the
  dimensionally consistent k_d h_d arguments).

Pins: tests/test_oracle_spectra.py compares every transform with adaptive
radial quadrature of its real-space definition, and the k -> 0 limits with the
printed values.
"""
import math

import mpmath as mp
import numpy as np
from scipy.special import spherical_jn

FOUR_PI = 4.0 * math.pi


def axis_k(n, h):
    """Wavenumbers of axis with n nodes and spacing h, eq. (Kvalues)."""
    j = np.arange(n)
    return np.where(j <= n / 2.0, 2.0 * math.pi * j / (n * h), -2.0 * math.pi * (n - j) / (n * h))


def axis_nyquist(n):
    """True on the index j = n/2 of an even axis (its own mirror image)."""
    j = np.arange(n)
    return (j * 2 == n) if n % 2 == 0 else np.zeros(n, bool)


class KMesh:
    """Full (not half) FFT mesh for arrays laid out [z][y][x]."""

    def __init__(self, n, h):
        nx, ny, nz = n
        self.kx = axis_k(nx, h[0])[None, None, :]
        self.ky = axis_k(ny, h[1])[None, :, None]
        self.kz = axis_k(nz, h[2])[:, None, None]
        self.k = np.sqrt(self.kx ** 2 + self.ky ** 2 + self.kz ** 2)
        self.comp = [self.kx, self.ky, self.kz]
        self.nyq = [axis_nyquist(nx)[None, None, :], axis_nyquist(ny)[None, :, None],
                    axis_nyquist(nz)[:, None, None]]
        self.h = tuple(h)
        self.n = tuple(n)


def weight_spectra(R, mesh: KMesh):
    """Transforms of the six FMT weights of a sphere of radius R (e^{-i k.x} convention).

    Returns dict with real arrays 'w0','w1','w2','w3' and lists 'wv1','wv2' of
    three complex arrays (x, y, z components).
    """
    k = mesh.k
    y = k * R
    j0 = spherical_jn(0, y)
    j1 = spherical_jn(1, y)
    w2 = FOUR_PI * R * R * j0
    with np.errstate(invalid="ignore", divide="ignore"):
        w3 = np.where(y > 0.0, FOUR_PI * R ** 3 * j1 / np.where(y > 0.0, y, 1.0), FOUR_PI * R ** 3 / 3.0)
        khat = [np.where(k > 0.0, c / np.where(k > 0.0, k, 1.0), 0.0) for c in mesh.comp]
    wv2 = []
    for d in range(3):
        comp = -1j * khat[d] * FOUR_PI * R * R * j1
        comp = np.where(mesh.nyq[d], 0.0, comp)
        wv2.append(comp)
    return {"w0": w2 / (FOUR_PI * R * R), "w1": w2 / (FOUR_PI * R), "w2": w2, "w3": w3,
            "wv1": [c / (FOUR_PI * R) for c in wv2], "wv2": wv2}


def _ball_moment_closed(nexp, R, k):
    """(4 pi / k) I_n(R, k) from the integration-by-parts closed forms (k > 0)."""
    y = k * R
    if nexp == -1:
        I = (1.0 - np.cos(y)) / k
    elif nexp == 0:
        I = -R / k * np.cos(y) + np.sin(y) / k ** 2
    elif nexp == 1:
        I = -R * R / k * np.cos(y) + 2.0 * R / k ** 2 * np.sin(y) - 2.0 / k ** 3 * (1.0 - np.cos(y))
    else:
        raise ValueError(nexp)
    return FOUR_PI / k * I


def _ball_moment_mp(nexp, R, k):
    with mp.workdps(40):
        R = mp.mpf(R)
        k = mp.mpf(k)
        c, s = mp.cos(k * R), mp.sin(k * R)
        if nexp == -1:
            I = (1 - c) / k
        elif nexp == 0:
            I = -R / k * c + s / k ** 2
        else:
            I = -R * R / k * c + 2 * R / k ** 2 * s - 2 / k ** 3 * (1 - c)
        return float(4 * mp.pi / k * I)


def ball_moment_limit(nexp, R):
    """Printed k -> 0 limits: 2 pi R^2, 4 pi R^3 / 3, pi R^4 for n = -1, 0, 1."""
    return {-1: 2.0 * math.pi * R ** 2, 0: FOUR_PI * R ** 3 / 3.0, 1: math.pi * R ** 4}[nexp]


def ball_moment(nexp, R, k):
    """integral over |r| <= R of r^n exp(-i k.r) d^3r = (4 pi / k) I_n, for an array of |k|."""
    k = np.asarray(k, float)
    out = np.empty(k.shape)
    small = k * R < 1.0
    big = ~small
    if np.any(big):
        out[big] = _ball_moment_closed(nexp, R, k[big])
    if np.any(small):
        ks = k[small]
        uniq, inv = np.unique(ks, return_inverse=True)
        vals = np.array([ball_moment_limit(nexp, R) if u == 0.0 else _ball_moment_mp(nexp, R, u)
                         for u in uniq])
        out[small] = vals[inv.reshape(ks.shape)]
    return out


def screening_kernel(k, zi, zj, lam_i, lam_j, Rij, lB):
    """Transform of the bulk-fluid kernel beta(c2 + psi)_ij restricted to |r| <= R_ij.

    In real space (eq. (CplusPsiFunc), energies in kT):
      (z_i z_j l_B / 2) [ r/(2 l_i l_j) - (l_i + l_j)/(l_i l_j) + ((l_i - l_j)^2/(2 l_i l_j) + 2)/r ].
    """
    ll = lam_i * lam_j
    return 0.5 * zi * zj * lB * (ball_moment(1, Rij, k) / (2.0 * ll)
                                 - (lam_i + lam_j) / ll * ball_moment(0, Rij, k)
                                 + ((lam_i - lam_j) ** 2 / (2.0 * ll) + 2.0) * ball_moment(-1, Rij, k))


def screening_kernel_real(r, zi, zj, lam_i, lam_j, Rij, lB):
    """Real-space bulk-fluid kernel (eq. (CplusPsiFunc)), zero beyond R_ij."""
    r = np.asarray(r, float)
    ll = lam_i * lam_j
    with np.errstate(divide="ignore"):
        val = 0.5 * zi * zj * lB * (r / (2.0 * ll) - (lam_i + lam_j) / ll
                                    + ((lam_i - lam_j) ** 2 / (2.0 * ll) + 2.0) / r)
    return np.where(r <= Rij, val, 0.0)


def poisson_denominator(mesh: KMesh):
    """Eigenvalues of minus the 7-point Laplacian on the periodic grid."""
    D = 0.0
    for d in range(3):
        D = D + 2.0 * (1.0 - np.cos(mesh.comp[d] * mesh.h[d])) / mesh.h[d] ** 2
    return D
