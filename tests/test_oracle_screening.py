"""Pins for oracle.screening (RFD screening operator, O(N^2)): the ball transform against the
Appendix B weight spectra, constant and two-valued radius fields against FFT convolutions,
invariants (uniform fields, linearity, reality)."""
import math

import numpy as np
import pytest

from oracle import screening, spectra


def _grid(n=(12, 8, 9), h=(0.1, 0.12, 0.09)):
    return n, h, (n[2], n[1], n[0])


def test_ball_is_the_normalized_w3_spectrum():
    # B(kR) = w3(k; R) / (4 pi R^3 / 3); w3 is pinned to radial quadrature in test_oracle_spectra.
    n, h, shape = _grid()
    mesh = spectra.KMesh(n, h)
    for R in (0.05, 0.3, 1.1):
        w3 = spectra.weight_spectra(R, mesh)["w3"]
        assert np.allclose(screening.ball(mesh.k * R), w3 / (4 * math.pi * R ** 3 / 3), rtol=1e-13, atol=1e-15)
    assert screening.ball(np.array([0.0]))[0] == 1.0
    # small-argument series 1 - t^2/10 + t^4/280
    t = np.array([1e-4, 1e-3, 1e-2])
    assert np.allclose(screening.ball(t), 1 - t ** 2 / 10 + t ** 4 / 280, rtol=1e-15)


def test_constant_radius_is_the_fft_convolution():
    n, h, shape = _grid()
    rng = np.random.default_rng(0)
    f = rng.uniform(0.0, 2.0, (2,) + shape)
    R = np.full(shape, 0.27)
    a = screening.reference(f, R, n, h)
    b = screening.convolution(f, 0.27, n, h)
    assert np.allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())


def test_two_radii_select_the_two_convolutions():
    n, h, shape = _grid()
    rng = np.random.default_rng(1)
    f = rng.uniform(0.0, 2.0, shape)
    R = np.where(rng.uniform(size=shape) < 0.4, 0.15, 0.42)
    a = screening.reference(f, R, n, h)
    c1 = screening.convolution(f, 0.15, n, h)
    c2 = screening.convolution(f, 0.42, n, h)
    want = np.where(R == 0.15, c1, c2)
    assert np.allclose(a, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_uniform_field_and_linearity():
    n, h, shape = _grid()
    rng = np.random.default_rng(2)
    R = rng.uniform(0.1, 0.5, shape)
    assert np.allclose(screening.reference(np.full(shape, 0.7), R, n, h), 0.7, rtol=1e-14, atol=0)
    f, g = rng.normal(size=shape), rng.normal(size=shape)
    lhs = screening.reference(2.0 * f - 3.0 * g, R, n, h)
    rhs = 2.0 * screening.reference(f, R, n, h) - 3.0 * screening.reference(g, R, n, h)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-13 * np.abs(rhs).max())


def test_ball_average_of_a_plane_wave():
    # For f = cos(k0 . x) on a mesh wavevector k0, f_ref(x) = B(|k0| R(x)) cos(k0 . x) exactly.
    n, h, shape = _grid()
    rng = np.random.default_rng(3)
    R = rng.uniform(0.1, 0.5, shape)
    jx, jy, jz = 2, 1, 3
    X = (np.arange(n[0]) * h[0])[None, None, :]
    Y = (np.arange(n[1]) * h[1])[None, :, None]
    Z = (np.arange(n[2]) * h[2])[:, None, None]
    k0 = [2 * math.pi * jx / (n[0] * h[0]), 2 * math.pi * jy / (n[1] * h[1]), 2 * math.pi * jz / (n[2] * h[2])]
    f = np.cos(k0[0] * X + k0[1] * Y + k0[2] * Z) * np.ones(shape)
    want = screening.ball(np.linalg.norm(k0) * R) * f
    assert np.allclose(screening.reference(f, R, n, h), want, rtol=0, atol=1e-13)


def test_reference_at_sampled_points_equals_the_full_evaluation():
    n, h, shape = _grid()
    rng = np.random.default_rng(4)
    f = rng.uniform(0.0, 2.0, (2,) + shape)
    R = rng.uniform(0.1, 0.5, shape)
    full = screening.reference(f, R, n, h)
    pts = [(0, 0, 0), (3, 5, 7), (8, 7, 11)]
    got = screening.reference_at(f, R, n, h, pts)
    for q, p in enumerate(pts):
        assert np.allclose(got[:, q], full[:, p[0], p[1], p[2]], rtol=0, atol=1e-13 * np.abs(full).max())
