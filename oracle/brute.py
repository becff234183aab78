"""Real-space evaluation of the discrete convolution operators, for tiny grids.

The method's convolutions (eq. (conv) with the analytic spectra of Appendix B)
are circulant operators on the periodic grid:

    n(x) = sum_m K[x - m] rho[m],     K[m] = N^-1 sum_k w_hat(k) exp(i k.x_m).

Here K is tabulated by direct summation over every mode k (no FFT), with the
phases k.x_m reduced exactly as 2 pi (j m mod N) / N per axis, and the sums over
m are taken literally.  Cost O(N^2): meant for grids of at most a few thousand
nodes.  It pins the FFT-based operators of the residual module (normalization,
sign convention, Nyquist handling) and the transpose used by the
back-convolution.
"""
import math

import numpy as np


def _signed(n):
    j = np.arange(n)
    return np.where(j <= n / 2.0, j, j - n)


def _phase_matrix(n):
    """exp(i k.x_m) for every (k, m) pair, k and m flattened in [z][y][x] order."""
    nx, ny, nz = n
    jz, jy, jx = np.meshgrid(_signed(nz), _signed(ny), _signed(nx), indexing="ij")
    mz, my, mx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    jz, jy, jx = jz.ravel(), jy.ravel(), jx.ravel()
    mz, my, mx = mz.ravel(), my.ravel(), mx.ravel()
    ang = (2.0 * math.pi * np.mod(np.outer(jx, mx), nx) / nx
           + 2.0 * math.pi * np.mod(np.outer(jy, my), ny) / ny
           + 2.0 * math.pi * np.mod(np.outer(jz, mz), nz) / nz)
    return np.exp(1j * ang)


def kernel(spec, n):
    """Real-space kernel K[m] of the spectrum `spec` (array on the full mesh)."""
    N = int(np.prod(n))
    P = _phase_matrix(n)
    K = (spec.ravel() @ P) / N
    if np.max(np.abs(K.imag)) > 1e-12 * max(np.max(np.abs(K.real)), 1e-300):
        raise AssertionError("kernel is not real")
    nx, ny, nz = n
    return K.real.reshape(nz, ny, nx)


def _offsets(n):
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return z.ravel(), y.ravel(), x.ravel()


def conv(K, f):
    """out[x] = sum_m K[x - m] f[m] (periodic), literally."""
    nz, ny, nx = K.shape
    z, y, x = _offsets((nx, ny, nz))
    Kd = K[np.mod(z[:, None] - z[None, :], nz), np.mod(y[:, None] - y[None, :], ny),
           np.mod(x[:, None] - x[None, :], nx)]
    return (Kd @ f.ravel()).reshape(K.shape)


def conv_t(K, f):
    """out[m] = sum_x K[x - m] f[x], the transpose of `conv`."""
    nz, ny, nx = K.shape
    z, y, x = _offsets((nx, ny, nz))
    Kd = K[np.mod(z[:, None] - z[None, :], nz), np.mod(y[:, None] - y[None, :], ny),
           np.mod(x[:, None] - x[None, :], nx)]
    return (Kd.T @ f.ravel()).reshape(K.shape)


def _kernels(setup, i):
    w = setup.w[i]
    specs = [w["w0"], w["w1"], w["w2"], w["w3"]] + list(w["wv1"]) + list(w["wv2"])
    return [kernel(s * np.ones(setup.shape), setup.n) for s in specs]


def weighted_densities(setup, rho):
    out = np.zeros((10,) + setup.shape)
    for i in range(setup.S):
        for a, K in enumerate(_kernels(setup, i)):
            out[a] += conv(K, rho[i])
    return out


def back_convolution(setup, dphi):
    c = np.zeros((setup.S,) + setup.shape)
    for i in range(setup.S):
        for a, K in enumerate(_kernels(setup, i)):
            c[i] -= conv_t(K, dphi[a])
    return c
