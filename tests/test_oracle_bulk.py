"""Pins for oracle.bulk (Appendix A): textbook closed forms and thermodynamic identities."""
import math

import numpy as np
import pytest

from oracle import bulk


@pytest.mark.parametrize("eta", [1e-5, 0.05, 0.2, 0.3, 0.4])
def test_one_component_py_closed_forms(eta):
    # Percus-Yevick compressibility route for one component (equal to scaled-particle theory):
    #   beta P / rho = (1 + eta + eta^2) / (1 - eta)^3
    #   beta mu_ex   = -ln(1 - eta) + eta (14 - 13 eta + 5 eta^2) / (2 (1 - eta)^3)
    sigma = 1.3
    rho = 6 * eta / (math.pi * sigma ** 3)
    bP = bulk.hs_pressure([rho], [sigma])
    mu = bulk.hs_mu([rho], [sigma])[0]
    assert bP == pytest.approx(rho * (1 + eta + eta ** 2) / (1 - eta) ** 3, rel=1e-13)
    assert mu == pytest.approx(-math.log(1 - eta) + eta * (14 - 13 * eta + 5 * eta ** 2)
                               / (2 * (1 - eta) ** 3), rel=1e-13, abs=1e-15)


def test_c1_state_values():
    # sigma = 1, eta = 0.2: rho = 0.381971863421, beta P = 0.925088106722, beta mu_ex = 2.488768551314
    rho = 6 * 0.2 / math.pi
    assert rho == pytest.approx(0.381971863421, abs=1e-12)
    assert bulk.hs_pressure([rho], [1.0]) == pytest.approx(0.925088106722, abs=1e-12)
    assert bulk.hs_mu([rho], [1.0])[0] == pytest.approx(2.488768551314, abs=1e-12)


def test_mixture_of_identical_species_reduces_to_one_component():
    rho = np.array([0.1, 0.05, 0.2])
    sig = np.array([0.9, 0.9, 0.9])
    mu = bulk.hs_mu(rho, sig)
    mu1 = bulk.hs_mu([rho.sum()], [0.9])[0]
    assert np.allclose(mu, mu1, rtol=1e-14)
    assert bulk.hs_pressure(rho, sig) == pytest.approx(bulk.hs_pressure([rho.sum()], [0.9]), rel=1e-14)


def test_mixture_gibbs_duhem():
    # d(beta P)/d rho_k = 1 + sum_j rho_j d(beta mu_ex_j)/d rho_k for every k (asymmetric sizes).
    rho = np.array([0.3, 0.8, 0.1])
    sig = np.array([1.0, 0.6, 1.4])
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-6 * rho[k]
        dP = (bulk.hs_pressure(rho + e, sig) - bulk.hs_pressure(rho - e, sig)) / (2 * e[k])
        dmu = (bulk.hs_mu(rho + e, sig) - bulk.hs_mu(rho - e, sig)) / (2 * e[k])
        assert dP == pytest.approx(1.0 + np.dot(rho, dmu), rel=1e-8)


@pytest.mark.parametrize("eta", [1e-6, 0.05, 0.2, 0.3, 0.45])
def test_one_component_bmcsl_is_carnahan_starling(eta):
    # Carnahan-Starling: beta P / rho = (1 + eta + eta^2 - eta^3) / (1 - eta)^3,
    # beta mu_ex = eta (8 - 9 eta + 3 eta^2) / (1 - eta)^3, beta f_ex / rho = eta (4 - 3 eta) / (1 - eta)^2.
    sigma = 0.8
    rho = 6 * eta / (math.pi * sigma ** 3)
    assert bulk.bmcsl_pressure([rho], [sigma]) == pytest.approx(
        rho * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3, rel=1e-13)
    assert bulk.bmcsl_mu([rho], [sigma])[0] == pytest.approx(
        eta * (8 - 9 * eta + 3 * eta ** 2) / (1 - eta) ** 3, rel=1e-9 if eta < 1e-3 else 1e-13)
    assert bulk.bmcsl_free_energy([rho], [sigma]) == pytest.approx(
        rho * eta * (4 - 3 * eta) / (1 - eta) ** 2, rel=1e-9 if eta < 1e-3 else 1e-13)


def test_bmcsl_mixture_thermodynamic_identities():
    # beta P = sum_i rho_i (1 + beta mu_ex_i) - beta f_ex, Gibbs-Duhem, and mu_i = d f_ex / d rho_i.
    rho = np.array([0.3, 0.8, 0.1])
    sig = np.array([1.0, 0.6, 1.4])
    mu = bulk.bmcsl_mu(rho, sig)
    assert bulk.bmcsl_pressure(rho, sig) == pytest.approx(
        np.sum(rho * (1 + mu)) - bulk.bmcsl_free_energy(rho, sig), rel=1e-13)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-6 * rho[k]
        dP = (bulk.bmcsl_pressure(rho + e, sig) - bulk.bmcsl_pressure(rho - e, sig)) / (2 * e[k])
        dmu = (bulk.bmcsl_mu(rho + e, sig) - bulk.bmcsl_mu(rho - e, sig)) / (2 * e[k])
        df = (bulk.bmcsl_free_energy(rho + e, sig) - bulk.bmcsl_free_energy(rho - e, sig)) / (2 * e[k])
        assert dP == pytest.approx(1.0 + np.dot(rho, dmu), rel=1e-8)
        assert df == pytest.approx(mu[k], rel=1e-8)
    # identical species reduce to one component
    same = np.array([0.9, 0.9, 0.9])
    assert np.allclose(bulk.bmcsl_mu(rho, same), bulk.bmcsl_mu([rho.sum()], [0.9])[0], rtol=1e-13)


@pytest.mark.parametrize("c,sigma", [(0.1, 0.3), (1.0, 0.425), (0.01, 0.2)])
def test_msa_gamma_restricted_primitive_closed_form(c, sigma):
    # Equal diameters, symmetric valences: eta_MSA = 0 and Gamma = (sqrt(1 + 2 kappa sigma) - 1) / (2 sigma).
    lB = 0.714871584
    rho = np.array([c, c]) * 0.602214076
    z = np.array([1.0, -1.0])
    kappa = math.sqrt(4 * math.pi * lB * np.sum(rho * z ** 2))
    g = bulk.msa_gamma(rho, [sigma, sigma], z, lB)
    assert g == pytest.approx((math.sqrt(1 + 2 * kappa * sigma) - 1) / (2 * sigma), rel=1e-14)


def test_msa_debye_limit_and_equation_residual():
    lB = 0.714871584
    z = np.array([2.0, 1.0, -1.0])
    sig = np.array([0.2, 0.2, 0.362])
    base = np.array([0.01, 0.1, 0.12]) * 0.602214076
    for scale in (1e-6, 1e-4):
        rho = base * scale
        kappa = math.sqrt(4 * math.pi * lB * np.sum(rho * z ** 2))
        g = bulk.msa_gamma(rho, sig, z, lB)
        assert g == pytest.approx(kappa / 2, rel=3 * kappa * sig.max())
        # Debye-Hueckel limiting law for the electrostatic chemical potential.
        mu = bulk.msa_mu_es(rho, sig, z, lB)
        assert np.allclose(mu, -z ** 2 * lB * kappa / 2, rtol=5 * kappa * sig.max())
    g = bulk.msa_gamma(base, sig, z, lB)
    assert abs(bulk.msa_equation(g, base, sig, z, lB)) < 1e-14 * g * g


def test_msa_no_charge_returns_zero():
    assert bulk.msa_gamma([0.1, 0.1], [0.3, 0.3], [0.0, 0.0], 0.7) == 0.0
    assert bulk.msa_gamma([0.1, 0.1], [0.3, 0.3], [1.0, -1.0], 0.0) == 0.0
