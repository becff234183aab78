"""Bulk (homogeneous) thermodynamics, Appendix A of the paper.

* Percus-Yevick (compressibility) / scaled-particle hard-sphere excess chemical
  potential, eq. (muHSBath), and pressure, eq. (HSPressure), in terms of the
  moments xi_n = (pi/6) sum_j rho_j sigma_j^n and Delta = 1 - xi_3.
* Mean spherical approximation screening parameter Gamma, eq. (Gamma), with the
  asymmetry parameter eta and Omega defined beside it.  The paper solves the
  implicit equation by Newton's method; the oracle brackets the root with
  scipy's Brent solver, which reaches the same root.
* MSA bulk electrostatic chemical potential (reporting only: it cancels in the
  bulk-fluid Euler-Lagrange exponent).
* Boublik-Mansoori-Carnahan-Starling-Leland (BMCSL) excess free energy, pressure
  and chemical potentials: the bulk thermodynamics of the White Bear functional
  (oracle.fmt), which replaces the Percus-Yevick bath when that functional is used.
  mu_i is the derivative of the free-energy density with respect to rho_i, written
  out by hand.

Units: lengths in any unit, densities in unit^-3, energies in kT.  e^2/(kT eps)
is written 4 pi l_B with l_B the Bjerrum length in the same unit.

Pins (tests/test_oracle_bulk.py): one-component PY closed forms (Carnahan-free
Percus-Yevick expressions in eta), restricted-primitive-model closed form for
Gamma, the Debye limit Gamma -> kappa/2, and the FMT bulk consistency checks in
the residual tests; BMCSL: one-component Carnahan-Starling closed forms,
P = sum rho mu - f, Gibbs-Duhem, and the White Bear functional's bulk derivative
(tests/test_oracle_fmt.py).
"""
import math

import numpy as np
from scipy.optimize import brentq


def moments(rho_b, sigma):
    """xi_n = (pi/6) sum_j rho_j sigma_j^n for n = 0..3 (Appendix A)."""
    rho_b = np.asarray(rho_b, float)
    sigma = np.asarray(sigma, float)
    return np.array([math.pi / 6.0 * np.sum(rho_b * sigma ** n) for n in range(4)])


def hs_pressure(rho_b, sigma):
    """beta P^HS_bath, eq. (HSPressure)."""
    xi = moments(rho_b, sigma)
    D = 1.0 - xi[3]
    return 6.0 / math.pi * (xi[0] / D + 3.0 * xi[1] * xi[2] / D ** 2 + 3.0 * xi[2] ** 3 / D ** 3)


def hs_mu(rho_b, sigma):
    """beta mu^HS_bath per species, eq. (muHSBath)."""
    sigma = np.asarray(sigma, float)
    xi = moments(rho_b, sigma)
    D = 1.0 - xi[3]
    bP = hs_pressure(rho_b, sigma)
    return (-math.log(D) + (3.0 * xi[2] * sigma + 3.0 * xi[1] * sigma ** 2) / D
            + 9.0 * xi[2] ** 2 * sigma ** 2 / (2.0 * D ** 2) + bP * math.pi * sigma ** 3 / 6.0)


def bmcsl_free_energy(rho_b, sigma):
    """Excess free-energy density beta f_ex of the BMCSL equation of state."""
    xi = moments(rho_b, sigma)
    D = 1.0 - xi[3]
    return 6.0 / math.pi * ((xi[2] ** 3 / xi[3] ** 2 - xi[0]) * math.log(D) + 3.0 * xi[1] * xi[2] / D
                            + xi[2] ** 3 / (xi[3] * D ** 2))


def bmcsl_pressure(rho_b, sigma):
    """beta P of the BMCSL equation of state (ideal part included)."""
    xi = moments(rho_b, sigma)
    D = 1.0 - xi[3]
    return 6.0 / math.pi * (xi[0] / D + 3.0 * xi[1] * xi[2] / D ** 2 + (3.0 - xi[3]) * xi[2] ** 3 / D ** 3)


def bmcsl_mu(rho_b, sigma):
    """beta mu_ex per species: d(beta f_ex)/d(rho_i) = sum_n d(beta f_ex)/d(xi_n) (pi/6) sigma_i^n."""
    sigma = np.asarray(sigma, float)
    xi = moments(rho_b, sigma)
    D = 1.0 - xi[3]
    lD = math.log(D)
    a0 = -lD
    a1 = 3.0 * xi[2] / D
    a2 = 3.0 * xi[1] / D + 3.0 * xi[2] ** 2 * (lD / xi[3] ** 2 + 1.0 / (xi[3] * D ** 2))
    a3 = (xi[0] / D + 3.0 * xi[1] * xi[2] / D ** 2
          + xi[2] ** 3 * (-2.0 * lD / xi[3] ** 3 - 1.0 / (xi[3] ** 2 * D) - 1.0 / (xi[3] ** 2 * D ** 2)
                          + 2.0 / (xi[3] * D ** 3)))
    return a0 + a1 * sigma + a2 * sigma ** 2 + a3 * sigma ** 3


def bath(functional, rho_b, sigma):
    """(beta mu_ex per species, beta P) of the uniform fluid of a hard-sphere functional."""
    if functional in ("rslt", "rosenfeld"):
        return hs_mu(rho_b, sigma), hs_pressure(rho_b, sigma)
    if functional == "whitebear":
        return bmcsl_mu(rho_b, sigma), bmcsl_pressure(rho_b, sigma)
    raise ValueError(f"unknown functional {functional!r}")


def msa_terms(gamma, rho_b, sigma, z):
    """(eta, Omega) of the MSA at a trial Gamma (Appendix A, definitions after eq. (Gamma))."""
    rho_b, sigma, z = (np.asarray(a, float) for a in (rho_b, sigma, z))
    D = 1.0 - moments(rho_b, sigma)[3]
    omega = 1.0 + math.pi / (2.0 * D) * np.sum(rho_b * sigma ** 3 / (1.0 + gamma * sigma))
    eta = math.pi / (2.0 * D) * np.sum(rho_b * sigma * z / (1.0 + gamma * sigma)) / omega
    return eta, omega


def msa_equation(gamma, rho_b, sigma, z, lB):
    """4 Gamma^2 - 4 pi l_B sum_j rho_j ((z_j - eta sigma_j^2)/(1 + Gamma sigma_j))^2, eq. (Gamma)."""
    rho_b, sigma, z = (np.asarray(a, float) for a in (rho_b, sigma, z))
    eta, _ = msa_terms(gamma, rho_b, sigma, z)
    s = np.sum(rho_b * ((z - eta * sigma ** 2) / (1.0 + gamma * sigma)) ** 2)
    return 4.0 * gamma ** 2 - 4.0 * math.pi * lB * s


def msa_gamma(rho_b, sigma, z, lB):
    """Root Gamma > 0 of eq. (Gamma).  Returns 0 when there is no charge (l_B = 0 or all z = 0)."""
    rho_b, sigma, z = (np.asarray(a, float) for a in (rho_b, sigma, z))
    kappa2 = 4.0 * math.pi * lB * np.sum(rho_b * z ** 2)
    if kappa2 <= 0.0:
        return 0.0
    hi = math.sqrt(kappa2)      # F(0) < 0; grow the bracket until F(hi) > 0
    while msa_equation(hi, rho_b, sigma, z, lB) <= 0.0:
        hi *= 2.0
    return brentq(msa_equation, 0.0, hi, args=(rho_b, sigma, z, lB), xtol=1e-300, rtol=1e-15,
                  maxiter=500)


def msa_mu_es(rho_b, sigma, z, lB):
    """beta mu^ES_bath per species (Appendix A), with e^2/(4 pi eps eps0 kT) = l_B."""
    rho_b, sigma, z = (np.asarray(a, float) for a in (rho_b, sigma, z))
    g = msa_gamma(rho_b, sigma, z, lB)
    eta, _ = msa_terms(g, rho_b, sigma, z)
    return -lB * (g * z ** 2 / (1.0 + g * sigma)
                  + eta * sigma * ((2.0 * z - eta * sigma ** 2) / (1.0 + g * sigma) + eta * sigma ** 2 / 3.0))
