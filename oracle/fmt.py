"""Hard-sphere free-energy density of fundamental measure theory, eq. (Phi).

The anti-symmetrized Rosenfeld form the paper prints ("rslt", the default)

  Phi = -n0 ln(1 - n3) + (n1 n2 - nV1.nV2) / (1 - n3)
        + n2^3 (1 - xi^2)^3 / (24 pi (1 - n3)^2),      xi^2 = nV2.nV2 / n2^2.

Weighted densities are stacked in the order
  0:n0 1:n1 2:n2 3:n3 4-6:nV1 (x,y,z) 7-9:nV2 (x,y,z).

Enforcing the bound |nV2| <= n2 (section on numerical stability, Appendix C) is
read as xi^2 <- min(xi^2, 1), with n2^2 floored at 1e-300 in the ratio, so the
last term and its derivatives vanish continuously where the bound is violated.

Two alternatives the paper allows in place of eq. (Phi) (its hard-sphere section
says the choice of functional leaves the numerical scheme unchanged) keep the
first two terms and replace the third by

  Phi3 = (n2^3 - 3 n2 nV2.nV2) f(n3) / (36 pi),

  "rosenfeld":  f = 3 / (2 (1 - n3)^2)             (Rosenfeld's original vector form)
  "whitebear":  f = (n3 + (1 - n3)^2 ln(1 - n3)) / (n3^2 (1 - n3)^2)
                                                    (White Bear; bulk = BMCSL, oracle.bulk)

with the same reading of the bound: nV2.nV2 <- min(nV2.nV2, n2^2) (xi^2 <- min(xi^2, 1)).
The White Bear factor loses digits to cancellation as n3 -> 0 (f -> 3/2); below
|n3| = 0.1 it is summed from its Taylor series f = sum_k (k+1)(k+3)/(k+2) n3^k.

The first derivatives are written out by hand from the expressions above.
Pins: tests/test_oracle_fmt.py checks them against complex-step derivatives of
`phi`, checks the bulk identities (excess pressure and chemical potential of
the uniform fluid reduce to the Percus-Yevick closed forms of Appendix A for
"rslt" and "rosenfeld", and to the Carnahan-Starling / BMCSL closed forms for
"whitebear"), the White Bear factor's series against its closed form where both
are accurate, and `hessian_vec` (complex step of the hand-written gradient)
against central differences.
"""
import math

import numpy as np

NALPHA = 10
_PI = math.pi
FUNCTIONALS = ("rslt", "rosenfeld", "whitebear")
_WB_SERIES_BELOW = 0.1
_WB_TERMS = 30


def _xi2(n2, v2):
    """Clamped xi^2, choosing branches by real part so complex steps pass through."""
    n2sq = n2 * n2
    den = np.where(np.real(n2sq) > 1e-300, n2sq, 1e-300)
    xi2 = v2 / den
    return np.where(np.real(xi2) < 1.0, xi2, 1.0 + 0.0 * xi2)


def wb_factor(n3, series_below=_WB_SERIES_BELOW):
    """White Bear f(n3) and f'(n3) (complex-step safe: branches on the real part)."""
    n3 = np.asarray(n3)
    small = np.abs(np.real(n3)) < series_below
    # Taylor series, summed by Horner's rule from the highest power
    f = np.zeros_like(n3, dtype=np.result_type(n3, 1.0))
    fp = np.zeros_like(f)
    for k in range(_WB_TERMS - 1, -1, -1):
        c = (k + 1.0) * (k + 3.0) / (k + 2.0)
        fp = fp * n3 + f           # derivative of the running polynomial
        f = f * n3 + c
    # closed form elsewhere (n3 replaced where the series is used, so no 0/0 is formed)
    x = np.where(small, 0.5, n3)
    y = 1.0 - x
    lg = np.log1p(-x)
    fc = (x + y * y * lg) / (x * x * y * y)
    fpc = -2.0 * lg / x ** 3 - (x * x - 5.0 * x + 2.0) / (x * x * y ** 3)
    return np.where(small, f, fc), np.where(small, fp, fpc)


def _third_factor(n3, functional):
    """f(n3) and f'(n3) of the alternative third term."""
    if functional == "rosenfeld":
        D = 1.0 - n3
        return 1.5 / D ** 2, 3.0 / D ** 3
    if functional == "whitebear":
        return wb_factor(n3)
    raise ValueError(f"unknown functional {functional!r}; expected one of {FUNCTIONALS}")


def _clamped_dot22(n2, dot22):
    """nV2.nV2 with the bound applied (n2^2 where xi^2 >= 1) and the clamp mask."""
    clamped = np.real(_xi2(n2, dot22)) >= 1.0
    return np.where(clamped, n2 * n2, dot22), clamped


def phi(n, functional="rslt"):
    """Free-energy density (in kT per volume) at every point; n has shape [10, ...]."""
    if functional != "rslt":
        return _phi_alt(n, functional)
    n0, n1, n2, n3 = n[0], n[1], n[2], n[3]
    v1 = n[4:7]
    v2 = n[7:10]
    D = 1.0 - n3
    dot12 = v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2]
    dot22 = v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]
    q = 1.0 - _xi2(n2, dot22)
    return -n0 * np.log(D) + (n1 * n2 - dot12) / D + n2 ** 3 * q ** 3 / (24.0 * _PI * D ** 2)


def _phi_alt(n, functional):
    n0, n1, n2, n3 = n[0], n[1], n[2], n[3]
    v1 = n[4:7]
    v2 = n[7:10]
    D = 1.0 - n3
    dot12 = v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2]
    dot22 = v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]
    g, _ = _clamped_dot22(n2, dot22)
    f, _ = _third_factor(n3, functional)
    return -n0 * np.log(D) + (n1 * n2 - dot12) / D + (n2 ** 3 - 3.0 * n2 * g) * f / (36.0 * _PI)


def _dphi_alt(n, functional):
    n0, n1, n2, n3 = n[0], n[1], n[2], n[3]
    v1 = n[4:7]
    v2 = n[7:10]
    D = 1.0 - n3
    dot12 = v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2]
    dot22 = v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]
    g, clamped = _clamped_dot22(n2, dot22)
    f, fp = _third_factor(n3, functional)
    out = np.empty(np.shape(n), dtype=np.result_type(n, 1.0))
    out[0] = -np.log(D)
    out[1] = n2 / D
    # d/dn2 of (n2^3 - 3 n2 g) f / (36 pi): g = nV2.nV2 is free of n2 unless clamped (g = n2^2)
    dn2 = np.where(clamped, -6.0 * n2 * n2, 3.0 * n2 * n2 - 3.0 * g)
    out[2] = n1 / D + dn2 * f / (36.0 * _PI)
    out[3] = n0 / D + (n1 * n2 - dot12) / D ** 2 + (n2 ** 3 - 3.0 * n2 * g) * fp / (36.0 * _PI)
    for d in range(3):
        out[4 + d] = -v2[d] / D
        dv = np.where(clamped, 0.0, -6.0 * n2 * v2[d])
        out[7 + d] = -v1[d] / D + dv * f / (36.0 * _PI)
    return out


def dphi(n, functional="rslt"):
    """The ten partial derivatives dPhi/dn_alpha, stacked like n."""
    if functional != "rslt":
        return _dphi_alt(n, functional)
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


def hessian_vec(n, dn, step=1e-30, functional="rslt"):
    """(d^2 Phi / dn dn) . dn by a complex step of `dphi` (no subtractive cancellation)."""
    return np.imag(dphi(n + 1j * step * dn, functional)) / step


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
