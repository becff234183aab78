"""Screening operator of the reference-fluid-density (RFD) electrostatics: the smoothing of
eq. (rhoRef) written as the per-point dot product of eq. (rhoRefKDotProduct) with the kernel
transform of eq. (screening-kernel-hat).  O(N^2): small grids only.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

For fields f_i on the periodic grid and a radius field R(x) > 0 (the local screening length
R_SC of the RFD section), every grid point x takes the average of f_i over the ball of radius
R(x) centred on x, evaluated spectrally:

  f_ref_i(x) = N^-1 sum_k f_hat_i(k) B(|k| R(x)) exp(i k.x),   B(t) = 3 j1(t) / t,  B(0) = 1,

with f_hat the unnormalized forward DFT and k the discrete set of eq. (Kvalues)
(oracle.spectra).  B is the transform of the normalized ball indicator, 3 (sin t - t cos t) / t^3.

Reading: the printed kernel transform carries exp(+i k.x) from shifting the ball to x; with the
paper's exp(-i k.x) forward transform that shift contributes exp(-i k.x), whose conjugate in
eq. (rhoRefKDotProduct) gives the exp(+i k.x) above, i.e. the ball average centred on x (the
only reading under which a constant R reduces to the ball convolution of eq. (rhoRef)).  The
eq. (rhoRefKDotProduct) integral over k becomes the discrete inverse transform sum.  The
weights alpha_i of eq. (rhoBarDef) enter linearly: callers pass alpha_i rho_i as f_i.

Pins (tests/test_oracle_screening.py): B against the Appendix B ball transform w3 / (4 pi R^3 / 3)
of oracle.spectra (pinned to quadrature there); a constant R equals the FFT convolution with B (a
different algorithm); a field that takes two radii equals the two FFT convolutions selected point
by point; a uniform field is unchanged; the operator is linear and real.
"""
import numpy as np
from scipy.special import spherical_jn

from . import spectra


def ball(t):
    """B(t) = 3 j1(t) / t, the transform of the unit-mean ball indicator at k R = t."""
    t = np.asarray(t, float)
    out = np.ones_like(t)
    pos = t > 0.0
    out[pos] = 3.0 * spherical_jn(1, t[pos]) / t[pos]
    return out


def reference(f, R, n, h, chunk=256):
    """f_ref for fields f [S, nz, ny, nx] (or [nz, ny, nx]) and radii R [nz, ny, nx]: the per-point
    dot product over all N wavevectors."""
    f = np.asarray(f, float)
    single = f.ndim == 3
    if single:
        f = f[None]
    R = np.asarray(R, float)
    mesh = spectra.KMesh(n, h)
    N = int(np.prod(f.shape[1:]))
    ks = np.stack(np.broadcast_arrays(mesh.kx, mesh.ky, mesh.kz), -1).reshape(-1, 3)
    kmag = mesh.k.ravel()
    nx, ny, nz = n
    X = (np.arange(nx) * h[0])[None, None, :]
    Y = (np.arange(ny) * h[1])[None, :, None]
    Z = (np.arange(nz) * h[2])[:, None, None]
    xs = np.stack(np.broadcast_arrays(X, Y, Z), -1).reshape(-1, 3)
    fh = np.fft.fftn(f, axes=(-3, -2, -1)).reshape(f.shape[0], -1)
    Rf = R.ravel()
    out = np.empty((f.shape[0], N))
    for s in range(0, N, chunk):
        e = np.exp(1j * (xs[s:s + chunk] @ ks.T))            # exp(i k.x) for this block of points
        kern = e * ball(Rf[s:s + chunk, None] * kmag[None, :])
        v = kern @ fh.T / N                                  # [points, S]
        out[:, s:s + chunk] = v.real.T
    out = out.reshape(f.shape)
    return out[0] if single else out


def reference_at(f, R, n, h, points):
    """f_ref at the listed grid points [(iz, iy, ix), ...] only: the same dot product, O(N) per point,
    for grids too large for `reference`.  Returns [S, len(points)] (or [len(points)])."""
    f = np.asarray(f, float)
    single = f.ndim == 3
    if single:
        f = f[None]
    mesh = spectra.KMesh(n, h)
    fh = np.fft.fftn(f, axes=(-3, -2, -1))
    out = np.empty((f.shape[0], len(points)))
    for q, (iz, iy, ix) in enumerate(points):
        phase = np.exp(1j * (mesh.kx * ix * h[0] + mesh.ky * iy * h[1] + mesh.kz * iz * h[2]))
        kern = phase * ball(mesh.k * R[iz, iy, ix])
        out[:, q] = (np.tensordot(fh, kern, axes=([1, 2, 3], [0, 1, 2])) / kern.size).real
    return out[0] if single else out


def convolution(f, R0, n, h):
    """Ball average with one radius R0 everywhere, by FFT (the constant-radius special case)."""
    f = np.asarray(f, float)
    mesh = spectra.KMesh(n, h)
    return np.fft.ifftn(np.fft.fftn(f, axes=(-3, -2, -1)) * ball(mesh.k * R0), axes=(-3, -2, -1)).real
