"""Pins for oracle.fmt: derivatives by complex step, bulk Percus-Yevick identities, Hessian."""
import math

import numpy as np
import pytest

from oracle import bulk, fmt


def _random_n(rng, npts, xi_big=False):
    n = np.empty((10, npts))
    n[2] = rng.uniform(0.5, 2.0, npts)
    n[0] = n[2] / (4 * math.pi * 0.25) * rng.uniform(0.8, 1.2, npts)
    n[1] = n[2] / (4 * math.pi * 0.5) * rng.uniform(0.8, 1.2, npts)
    n[3] = rng.uniform(0.01, 0.6, npts)
    v2 = rng.normal(size=(3, npts))
    scale = rng.uniform(0.05, 0.95 if not xi_big else 1.5, npts) * n[2] / np.linalg.norm(v2, axis=0)
    n[7:10] = v2 * scale
    n[4:7] = n[7:10] / (4 * math.pi * 0.5) + 0.01 * rng.normal(size=(3, npts))
    return n


@pytest.mark.parametrize("xi_big", [False, True])
def test_dphi_matches_complex_step(xi_big):
    rng = np.random.default_rng(1)
    n = _random_n(rng, 200, xi_big)
    d = fmt.dphi(n)
    for a in range(10):
        e = np.zeros_like(n)
        e[a] = 1e-30
        cs = np.imag(fmt.phi(n + 1j * e)) / 1e-30
        assert np.allclose(d[a], cs, rtol=1e-13, atol=1e-13 * np.abs(cs).max() + 1e-300), a


def test_clamp_zeroes_the_tensor_term():
    rng = np.random.default_rng(2)
    n = _random_n(rng, 50)
    n[7:10] *= 3.0 * n[2] / np.linalg.norm(n[7:10], axis=0)   # |nV2| = 3 n2 > n2
    D = 1 - n[3]
    ref = -n[0] * np.log(D) + (n[1] * n[2] - np.sum(n[4:7] * n[7:10], axis=0)) / D
    assert np.allclose(fmt.phi(n), ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("rho,R", [([0.38197186342], [0.5]), ([0.02, 0.05, 0.01], [0.1, 0.1, 0.181]),
                                   ([0.3, 0.1], [0.5, 0.3])])
def test_bulk_fmt_reproduces_percus_yevick(rho, R):
    # Uniform fluid: c_i = -sum_alpha dPhi/dn_alpha w_hat_alpha^i(0) must equal -beta mu_PY_i, and
    # n0 + sum_alpha n_alpha dPhi_alpha - Phi must equal beta P_PY (Appendix A closed forms).
    rho, R = np.asarray(rho), np.asarray(R)
    n = fmt.bulk_weighted(rho, R)
    d = fmt.dphi(n[:, None])[:, 0]
    mu = np.array([d[0] + d[1] * Ri + d[2] * 4 * math.pi * Ri ** 2 + d[3] * 4 * math.pi * Ri ** 3 / 3
                   for Ri in R])
    assert np.allclose(mu, bulk.hs_mu(rho, 2 * R), rtol=1e-13)
    P = n[0] + np.dot(n, d) - fmt.phi(n[:, None])[0]
    assert P == pytest.approx(bulk.hs_pressure(rho, 2 * R), rel=1e-13)


def test_fundamental_measures_c1():
    n = fmt.bulk_weighted([0.381971863421], [0.5])
    assert n[0] == pytest.approx(0.381971863421, abs=1e-12)
    assert n[1] == pytest.approx(0.190985931710, abs=1e-12)
    assert n[2] == pytest.approx(1.2, abs=1e-11)
    assert n[3] == pytest.approx(0.2, abs=1e-12)


def test_hessian_vec_against_central_difference():
    rng = np.random.default_rng(3)
    n = _random_n(rng, 100)
    dn = rng.normal(size=n.shape) * 1e-2 * np.abs(n).max(axis=1, keepdims=True)
    hv = fmt.hessian_vec(n, dn)
    eps = 1e-6
    fd = (fmt.dphi(n + eps * dn) - fmt.dphi(n - eps * dn)) / (2 * eps)
    assert np.allclose(hv, fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())
    # symmetry of the Hessian: u . H v = v . H u
    du = rng.normal(size=n.shape) * 1e-2
    assert np.allclose(np.sum(du * fmt.hessian_vec(n, dn), axis=0),
                       np.sum(dn * fmt.hessian_vec(n, du), axis=0), rtol=1e-10, atol=1e-14)
