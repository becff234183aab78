"""Pins for oracle.residual: invariants the paper and the mathematics fix."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import brute, fmt, residual, spectra


def _mixture(n=(6, 4, 5), h=(0.11, 0.13, 0.09)):
    p = W.Problem(name="mix", n=n, h=h, radius=np.array([0.21, 0.14]), valence=np.array([1.0, -1.0]),
                  rho_bulk=np.array([0.8, 1.1]), bjerrum=0.3, electrostatics=True)
    return p


def test_fundamental_measures_from_uniform_density():
    # Verification section: a constant density recovers the fundamental measures; bath n3 = packing.
    p = W.config_hs_wall()
    p.beta_vext = None
    st = residual.Setup(p)
    n = st.weighted_densities(p.initial_density())
    rho = 6 * 0.2 / math.pi          # sigma = 1, eta = 0.2
    exp = [rho, 0.5 * rho, 4 * math.pi * 0.25 * rho, 0.2]   # sum rho, sum rho R, 4 pi sum rho R^2, eta
    assert exp[0] == pytest.approx(0.381971863421, abs=1e-12) and exp[2] == pytest.approx(1.2, abs=1e-14)
    for a in range(4):
        assert np.allclose(n[a], exp[a], rtol=1e-14, atol=0)
    assert np.abs(n[4:]).max() < 1e-15


@pytest.mark.parametrize("n", [(6, 4, 5), (4, 4, 4), (3, 1, 1), (8, 2, 1)])
def test_fft_operators_equal_real_space_sums(n):
    p = _mixture(n=n)
    st = residual.Setup(p)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.2, 1.0, (2,) + st.shape)
    na = st.weighted_densities(rho)
    nb = brute.weighted_densities(st, rho)
    assert np.allclose(na, nb, rtol=0, atol=2e-14 * np.abs(nb).max())
    u = rng.normal(size=(10,) + st.shape)
    ca = st.back_convolution(u)
    cb = brute.back_convolution(st, u)
    assert np.allclose(ca, cb, rtol=0, atol=2e-14 * np.abs(cb).max())


def test_c_hs_is_minus_the_gradient_of_the_free_energy():
    # c_HS = -h^-3 dF/drho with F = h^3 sum_x Phi(n(x)): pins signs, transposition and Nyquist handling.
    p = _mixture(n=(6, 4, 4))
    st = residual.Setup(p)
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.3, 0.9, (2,) + st.shape) * 0.4
    c = st.back_convolution(fmt.dphi(st.weighted_densities(rho)))
    vol = float(np.prod(st.h))
    for _ in range(6):
        i = rng.integers(0, 2)
        idx = tuple(rng.integers(0, s) for s in st.shape)
        e = np.zeros_like(rho)
        e[(i,) + idx] = 1e-5
        dF = (st.free_energy_hs(rho + e) - st.free_energy_hs(rho - e)) / 2e-5
        assert c[(i,) + idx] == pytest.approx(-dF / vol, rel=1e-7, abs=1e-9)


def test_poisson_solution_satisfies_the_stencil():
    p = _mixture(n=(6, 4, 5))
    st = residual.Setup(p)
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.2, 1.0, (2,) + st.shape)
    phi = st.potential(rho)
    q = p.valence[0] * rho[0] + p.valence[1] * rho[1]
    lap = 0
    for ax, hd in ((2, p.h[0]), (1, p.h[1]), (0, p.h[2])):
        lap = lap + (np.roll(phi, 1, ax) + np.roll(phi, -1, ax) - 2 * phi) / hd ** 2
    rhs = 4 * math.pi * p.bjerrum * (q - q.mean())
    assert np.allclose(-lap, rhs, rtol=0, atol=1e-12 * np.abs(rhs).max())
    assert abs(phi.mean()) < 1e-14 * np.abs(phi).max()


def test_screening_acts_as_its_symbol_on_a_plane_wave():
    p = _mixture(n=(8, 6, 5))
    st = residual.Setup(p)
    jx, jy, jz = 2, 1, 3
    x = [np.arange(p.n[d]) * p.h[d] for d in range(3)]
    k = [st.mesh.kx[0, 0, jx], st.mesh.ky[0, jy, 0], st.mesh.kz[jz, 0, 0]]
    wave = np.cos(k[2] * x[2][:, None, None] + k[1] * x[1][None, :, None] + k[0] * x[0][None, None, :])
    rho = np.stack([p.rho_bulk[0] + 0.1 * wave, p.rho_bulk[1] + 0 * wave])
    c = st.screening(residual.dft(rho))
    kk = math.sqrt(sum(v * v for v in k))
    for i in range(2):
        Rij = p.radius[i] + p.radius[0]
        sym = spectra.screening_kernel(np.array([kk]), p.valence[i], p.valence[0], st.lam[i], st.lam[0],
                                       Rij, p.bjerrum)[0]
        assert np.allclose(c[i], sym * 0.1 * wave, rtol=0, atol=1e-14)


@pytest.mark.parametrize("es", [False, True])
def test_bulk_is_a_fixed_point(es):
    p = W.charged_pore(n=8, h=0.1) if es else W.hard_wall(n=(8, 8, 8), h=0.2, eta=0.3)
    p.beta_vext = None
    p.fixed_charge = None
    st = residual.Setup(p)
    rho = p.initial_density()
    G = st.G(rho)
    assert np.allclose(G, rho, rtol=1e-14, atol=0)


def test_planar_problem_is_homogeneous_and_matches_1d():
    p3 = W.hard_wall(n=(20, 4, 6), h=0.2, eta=0.25)
    p1 = W.hard_wall(n=(20, 1, 1), h=0.2, eta=0.25)
    st3, st1 = residual.Setup(p3), residual.Setup(p1)
    rng = np.random.default_rng(5)
    prof = p1.initial_density() * (1 + 0.3 * rng.uniform(-1, 1, (1, 1, 1, 20)))
    rho3 = np.broadcast_to(prof, (1, 6, 4, 20)).copy()
    G3, G1 = st3.G(rho3), st1.G(prof)
    assert np.abs(G3 - G3[:, :1, :1, :]).max() <= 1e-14 * G3.max()
    assert np.allclose(G3[:, 0, 0, :], G1[:, 0, 0, :], rtol=1e-13, atol=0)


def test_mirror_symmetry_of_the_residual():
    # Reflecting the density through x -> -x reflects G: the vector weights' signs are consistent.
    p = _mixture(n=(8, 4, 5))
    st = residual.Setup(p)
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.05, 0.3, (2,) + st.shape)
    G = st.G(rho)
    flip = lambda a: np.roll(a[..., ::-1], 1, axis=-1)
    assert np.allclose(st.G(flip(rho)), flip(G), rtol=1e-12, atol=0)
