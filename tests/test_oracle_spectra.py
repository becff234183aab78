"""Pins for oracle.spectra: quadrature of the real-space definitions, printed limits, symmetry."""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import spectra

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_limits.json")


def test_axis_k_ordering_even_and_odd():
    h = 0.3
    assert np.allclose(spectra.axis_k(4, h), 2 * math.pi / (4 * h) * np.array([0, 1, 2, -1]))
    assert np.allclose(spectra.axis_k(5, h), 2 * math.pi / (5 * h) * np.array([0, 1, 2, -2, -1]))
    assert np.allclose(spectra.axis_k(1, h), [0.0])
    assert list(spectra.axis_nyquist(4)) == [False, False, True, False]
    assert not spectra.axis_nyquist(5).any()


class _Mesh1:
    """A mesh whose |k| runs over chosen values along x (for quadrature comparisons)."""

    def __init__(self, ks):
        self.kx = np.asarray(ks, float)[None, None, :]
        self.ky = np.zeros((1, 1, 1))
        self.kz = np.zeros((1, 1, 1))
        self.k = np.abs(self.kx) + 0 * self.ky
        self.comp = [self.kx, self.ky, self.kz]
        self.nyq = [np.zeros_like(self.kx, bool), np.zeros((1, 1, 1), bool), np.zeros((1, 1, 1), bool)]


KS = [1e-7, 1e-4, 0.01, 0.3, 1.0, 2.7, 9.0, 31.0]


def test_weight_spectra_against_quadrature():
    R = 0.37
    w = spectra.weight_spectra(R, _Mesh1(KS))
    for i, k in enumerate(KS):
        # shell: integral of exp(-i k R cos t) over the sphere of radius R
        re = quad(lambda t: 2 * math.pi * R * R * math.sin(t) * math.cos(k * R * math.cos(t)), 0, math.pi,
                  epsabs=1e-15, epsrel=1e-13)[0]
        # ball: 4 pi int r^2 sin(kr)/(kr) dr
        vol = quad(lambda r: 4 * math.pi * r * r * np.sinc(k * r / math.pi), 0, R, epsabs=1e-15, epsrel=1e-13)[0]
        # vector shell (x component, k along x): -i int R^2 cos t sin(kR cos t) dOmega
        vx = -quad(lambda t: 2 * math.pi * R * R * math.sin(t) * math.cos(t) * math.sin(k * R * math.cos(t)),
                   0, math.pi, epsabs=1e-17, epsrel=1e-12)[0]
        assert w["w2"][0, 0, i] == pytest.approx(re, rel=1e-12)
        assert w["w0"][0, 0, i] == pytest.approx(re / (4 * math.pi * R * R), rel=1e-12)
        assert w["w1"][0, 0, i] == pytest.approx(re / (4 * math.pi * R), rel=1e-12)
        assert w["w3"][0, 0, i] == pytest.approx(vol, rel=1e-12)
        assert w["wv2"][0][0, 0, i].real == 0.0
        assert w["wv2"][0][0, 0, i].imag == pytest.approx(vx, rel=1e-10, abs=1e-22)
        assert w["wv1"][0][0, 0, i].imag == pytest.approx(vx / (4 * math.pi * R), rel=1e-10, abs=1e-22)


def test_weight_spectra_printed_k0_limits():
    g = json.load(open(GOLDEN))
    R = g["radius"]
    w = spectra.weight_spectra(R, _Mesh1([0.0]))
    for key in ("w0", "w1", "w2", "w3"):
        assert w[key][0, 0, 0] == pytest.approx(g["omega_hat_k0"][key], rel=1e-15)
    for d in range(3):
        assert w["wv1"][d][0, 0, 0] == 0 and w["wv2"][d][0, 0, 0] == 0


@pytest.mark.parametrize("nexp", [-1, 0, 1])
def test_ball_moments_against_quadrature_and_limits(nexp):
    R = 0.5
    ks = np.array([1e-6, 1e-3, 0.2, 1.5, 2.0, 7.0, 40.0])
    got = spectra.ball_moment(nexp, R, ks)
    for k, v in zip(ks, got):
        ref = 4 * math.pi / k * quad(lambda r: r ** (nexp + 1) * math.sin(k * r), 0, R, epsabs=1e-18,
                                     epsrel=1e-13, limit=200)[0]
        assert v == pytest.approx(ref, rel=1e-11)
    g = json.load(open(GOLDEN))
    assert spectra.ball_moment(nexp, g["radius"], np.array([0.0]))[0] == \
        pytest.approx(g["ball_moment_k0"][str(nexp)], rel=1e-15)


def test_screening_kernel_against_radial_quadrature():
    lB, zi, zj = 0.714871584, 2.0, -1.0
    Ri, Rj, gamma = 0.1, 0.181, 0.519681777037
    li, lj = Ri + 0.5 / gamma, Rj + 0.5 / gamma
    Rij = Ri + Rj
    for k in [0.0, 1e-5, 0.9, 3.3, 12.0, 60.0]:
        def integrand(r):
            s = np.sinc(k * r / math.pi)
            return 4 * math.pi * r * r * spectra.screening_kernel_real(r, zi, zj, li, lj, Rij, lB) * s
        ref = quad(integrand, 0, Rij, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
        got = spectra.screening_kernel(np.array([k]), zi, zj, li, lj, Rij, lB)[0]
        assert got == pytest.approx(ref, rel=1e-11)


def test_screening_kernel_small_r_is_coulomb():
    # beta(c2 + psi) -> z_i z_j l_B / r as r -> 0 (for equal lambdas the bracket's 1/r coefficient is 2).
    lB = 0.7
    r = 1e-9
    v = spectra.screening_kernel_real(r, 1.0, -1.0, 1.2, 1.2, 0.3, lB)
    assert v * r == pytest.approx(-lB, rel=1e-8)


def test_mesh_spectra_hermitian_and_nyquist():
    n, h = (6, 4, 5), (0.1, 0.13, 0.08)
    mesh = spectra.KMesh(n, h)
    w = spectra.weight_spectra(0.21, mesh)

    def mirror(a):
        a = np.broadcast_to(a, (n[2], n[1], n[0]))
        return np.roll(a[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))

    for key in ("w0", "w1", "w2", "w3"):
        a = np.broadcast_to(w[key], (5, 4, 6))
        assert np.allclose(mirror(a), a, rtol=0, atol=1e-15 * np.abs(a).max())
    for d in range(3):
        a = np.broadcast_to(w["wv2"][d], (5, 4, 6))
        assert np.allclose(mirror(a), np.conj(a), rtol=0, atol=1e-15 * np.abs(a).max())
    # component x is zero on the x Nyquist plane (n_x = 6: j = 3)
    assert np.all(np.broadcast_to(w["wv2"][0], (5, 4, 6))[:, :, 3] == 0)


def test_poisson_denominator_is_the_7_point_stencil_symbol():
    n, h = (8, 6, 5), (0.1, 0.2, 0.07)
    mesh = spectra.KMesh(n, h)
    D = spectra.poisson_denominator(mesh)
    x = [np.arange(n[d]) * h[d] for d in range(3)]
    rng = np.random.default_rng(0)
    for _ in range(5):
        jx, jy, jz = rng.integers(0, n[0]), rng.integers(0, n[1]), rng.integers(0, n[2])
        kx, ky, kz = mesh.kx[0, 0, jx], mesh.ky[0, jy, 0], mesh.kz[jz, 0, 0]
        f = np.exp(1j * (kz * x[2][:, None, None] + ky * x[1][None, :, None] + kx * x[0][None, None, :]))
        lap = 0
        for ax, hd in ((2, h[0]), (1, h[1]), (0, h[2])):
            lap = lap + (np.roll(f, 1, ax) + np.roll(f, -1, ax) - 2 * f) / hd ** 2
        assert np.allclose(-lap, D[jz, jy, jx] * f, atol=1e-9 * abs(D[jz, jy, jx]) + 1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_screening_bracket_double_zero_at_lambda_sum(seed):
    # The bulk-fluid kernel of eq. (CplusPsiFunc) must end smoothly where the MSA pair function
    # c^(2) + beta psi ends, at r = lambda_i + lambda_j: value and slope vanish there.  r times
    # the bracket is a quadratic in r (its linear, constant and 1/r coefficients become the
    # r^2, r and constant ones), so a degree-4 fit through five samples of the oracle's kernel
    # recovers it exactly; a dropped term or a wrong sign in any coefficient moves the double
    # root.  Together with the Coulomb limit at equal lambdas this fixes all three coefficients.
    rng = np.random.default_rng(seed)
    lam_i, lam_j = rng.uniform(0.2, 1.5, 2)
    lB, zi, zj = 0.714871584, float(rng.choice([1.0, 2.0])), -1.0
    L = lam_i + lam_j
    pref = 0.5 * zi * zj * lB
    r = np.linspace(0.3 * L, 1.7 * L, 5)
    g = r * spectra.screening_kernel_real(r, zi, zj, lam_i, lam_j, 10.0 * L, lB) / pref
    c = np.polynomial.polynomial.polyfit(r / L, g, 4)      # powers of r / L
    scale = np.max(np.abs(g))
    assert abs(c[3]) < 1e-12 * scale and abs(c[4]) < 1e-12 * scale
    poly = np.polynomial.Polynomial(c)
    assert abs(poly(1.0)) < 1e-13 * scale                # bracket zero at r = lambda_i + lambda_j
    assert abs(poly.deriv()(1.0)) < 1e-13 * scale        # and its r-derivative
    # past the double root the bracket stays of one sign (a minimum of |bracket|, not a crossing)
    rr = np.linspace(0.5 * L, 1.5 * L, 101)
    b = spectra.screening_kernel_real(rr, zi, zj, lam_i, lam_j, 10.0 * L, lB) / pref
    assert np.all(b >= -1e-14 * np.max(np.abs(b)))
