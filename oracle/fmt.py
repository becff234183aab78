"""Hard-sphere free-energy density of fundamental measure theory, eq. (Phi).

The anti-symmetrized Rosenfeld form

  Phi = -n0 ln(1 - n3) + (n1 n2 - nV1.nV2) / (1 - n3)
        + n2^3 (1 - xi^2)^3 / (24 pi (1 - n3)^2),      xi^2 = nV2.nV2 / n2^2.

Weighted densities are stacked in the order
  0:n0 1:n1 2:n2 3:n3 4-6:nV1 (x,y,z) 7-9:nV2 (x,y,z).

Enforcing the bound |nV2| <= n2 (section on numerical stability, Appendix C) is
read as xi^2 <- min(xi^2, 1), with n2^2 floored at 1e-300 in the ratio, so the
last term and its derivatives vanish continuously where the bound is violated.

The first derivatives are written out by hand from the expression above.
Pins: tests/test_oracle_fmt.py checks them against complex-step derivatives of
`phi`, checks the bulk identities (excess pressure and chemical potential of
the uniform fluid reduce to the Percus-Yevick closed forms of Appendix A), and
`hessian_vec` (complex step of the hand-written gradient) against central
differences.
"""
import math

import numpy as np

NALPHA = 10
_PI = math.pi


def _xi2(n2, v2):
    """Clamped xi^2, choosing branches by real part so complex steps pass through."""
    n2sq = n2 * n2
    den = np.where(np.real(n2sq) > 1e-300, n2sq, 1e-300)
    xi2 = v2 / den
    return np.where(np.real(xi2) < 1.0, xi2, 1.0 + 0.0 * xi2)


def phi(n):
    """Free-energy density (in kT per volume) at every point; n has shape [10, ...]."""
    n0, n1, n2, n3 = n[0], n[1], n[2], n[3]
    v1 = n[4:7]
    v2 = n[7:10]
    D = 1.0 - n3
    dot12 = v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2]
    dot22 = v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]
    q = 1.0 - _xi2(n2, dot22)
    return -n0 * np.log(D) + (n1 * n2 - dot12) / D + n2 ** 3 * q ** 3 / (24.0 * _PI * D ** 2)


def dphi(n):
    """The ten partial derivatives dPhi/dn_alpha, stacked like n."""
    n0, n1, n2, n3 = n[0], n[1], n[2], n[3]
    v1 = n[4:7]
    v2 = n[7:10]
    D = 1.0 - n3
    dot12 = v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2]
    dot22 = v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]
    x2 = _xi2(n2, dot22)
    q = 1.0 - x2
    out = np.empty(np.shape(n), dtype=np.result_type(n, 1.0))
    out[0] = -np.log(D)
    out[1] = n2 / D
    out[2] = n1 / D + n2 * n2 * q * q * (1.0 + x2) / (8.0 * _PI * D * D)
    out[3] = n0 / D + (n1 * n2 - dot12) / D ** 2 + n2 ** 3 * q ** 3 / (12.0 * _PI * D ** 3)
    for d in range(3):
        out[4 + d] = -v2[d] / D
        out[7 + d] = -v1[d] / D - n2 * q * q * v2[d] / (4.0 * _PI * D * D)
    return out


def hessian_vec(n, dn, step=1e-30):
    """(d^2 Phi / dn dn) . dn by a complex step of `dphi` (no subtractive cancellation)."""
    return np.imag(dphi(n + 1j * step * dn)) / step


def bulk_weighted(rho_b, R):
    """Weighted densities of a uniform fluid: the fundamental measures (vector parts zero)."""
    rho_b = np.asarray(rho_b, float)
    R = np.asarray(R, float)
    n = np.zeros(NALPHA)
    n[0] = np.sum(rho_b)
    n[1] = np.sum(rho_b * R)
    n[2] = np.sum(rho_b * 4.0 * _PI * R ** 2)
    n[3] = np.sum(rho_b * 4.0 * _PI * R ** 3 / 3.0)
    return n
