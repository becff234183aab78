"""One residual evaluation G(rho) of the Euler-Lagrange fixed point, plain FP64.

Steps, in the paper's order (theory section, hard-sphere and electrostatics
sections, discretization section):

  R1  rho_hat_i = DFT(rho_i)                          eq. (conv), FFT of each species
  R2  n_alpha  = IDFT(sum_i rho_hat_i w_hat_alpha^i)  eqs. (nDef), (conv); Appendix B spectra
  R3  dPhi/dn_alpha pointwise                         eq. (Phi)
  R4  c_HS_i = -sum_alpha IDFT(DFT(dPhi_alpha) conj(w_hat_alpha^i))     eq. (muHS), c = -beta mu
  R5  beta e phi_hat = 4 pi l_B (sum_j z_j rho_hat_j + q_hat)/D(k), phi_hat(0) = 0
                                                      eqs. (Poisson), (potentialSolution),
                                                      (potentialConstraint)
  R6  c_SC_i = sum_j IDFT(C_hat_ij (rho_hat_j - N rho_b_j delta_k0))    eq. (muESexpansion)
  R7  E_i = c_HS_i + c_SC_i - z_i beta e phi
  R8  G_i = rho_b_i exp(beta mu_HS_bath_i - beta V_i + E_i) on fluid nodes, 0 elsewhere
                                                      eq. (rhoEquation) with the bath
                                                      chemical potential of Appendix A
                                                      (BMCSL for the White Bear functional)

Readings (the paper is silent or ambiguous):
  * DFT is unnormalized with exp(-i k.x); IDFT carries 1/N, so the discrete
    convolution with a transform w_hat has kernel N^-1 sum_k w_hat e^{ik.x}.
  * The forward weighted densities multiply by w_hat; the back-convolution is
    the exact transpose (multiply by conj(w_hat)).  The vector sign convention
    of eq. (nDef) then cancels: Phi sees vectors only through dot products.
  * mu^ES_bath cancels between mu_bath and mu^SC in the bulk-fluid exponent,
    so G uses only the hard-sphere bath potential.
  * The screening kernel is cut at R_ij = R_i + R_j as printed.
  * Fixed charges (e.g. a charged sphere or pore sites) enter the Poisson
    source only.
  * All convolutions use scipy.fft in FP64 (a library primitive); the brute
    module evaluates the same circulant operators in real space to pin them.
"""
import math
import os

import numpy as np
import scipy.fft as sfft

from . import bulk, fmt, spectra

_WORKERS = max(1, len(os.sched_getaffinity(0)))


def dft(f):
    return sfft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def idft(F):
    return sfft.ifftn(F, axes=(-3, -2, -1), workers=_WORKERS)


def _real(F, what, check=True):
    f = idft(F)
    if check:
        scale = max(np.max(np.abs(f.real)), 1e-300)
        bad = np.max(np.abs(f.imag)) / scale
        if bad > 1e-12:
            raise AssertionError(f"{what}: imaginary part {bad:.2e} of the real part")
    return f.real


class Setup:
    """Everything computed once per problem (discretization section: setup-time work)."""

    def __init__(self, prob, cutoff="contact"):
        self.prob = prob
        self.S = prob.nspecies
        self.n = tuple(prob.n)
        self.h = tuple(prob.h)
        self.shape = prob.shape
        self.N = int(np.prod(self.shape))
        self.R = np.asarray(prob.radius, float)
        self.z = np.asarray(prob.valence, float)
        self.rho_b = np.asarray(prob.rho_bulk, float)
        self.lB = float(prob.bjerrum)
        self.es = bool(prob.electrostatics) and self.lB > 0.0
        self.eta_cap = float(prob.eta_cap)
        sigma = 2.0 * self.R
        self.functional = getattr(prob, "hs_functional", "rslt")
        self.mu_hs, self.betaP = bulk.bath(self.functional, self.rho_b, sigma)
        self.mesh = spectra.KMesh(self.n, self.h)
        self.w = [spectra.weight_spectra(R, self.mesh) for R in self.R]
        if prob.beta_vext is None:
            bv = np.zeros((self.S,) + self.shape)
        else:
            bv = np.asarray(prob.beta_vext, float)
        self.mask = np.isfinite(bv)
        self.vext = np.where(self.mask, bv, 0.0)
        self.nfluid = int(np.sum(self.mask))
        self.gamma = 0.0
        if self.es:
            self.gamma = bulk.msa_gamma(self.rho_b, sigma, self.z, self.lB)
            self.lam = self.R + 0.5 / self.gamma
            self.D = spectra.poisson_denominator(self.mesh)
            self.Chat = [[None] * self.S for _ in range(self.S)]
            for i in range(self.S):
                for j in range(i, self.S):
                    Rij = self.R[i] + self.R[j]
                    if cutoff == "lambda":
                        Rij = self.lam[i] + self.lam[j]
                    C = spectra.screening_kernel(self.mesh.k, self.z[i], self.z[j], self.lam[i],
                                                 self.lam[j], Rij, self.lB)
                    self.Chat[i][j] = self.Chat[j][i] = C
            q = prob.fixed_charge
            self.qhat = dft(q) if q is not None else None

    # ------------------------------------------------------------------ operators
    def weighted_densities(self, rho, rho_hat=None, check=True):
        """R1-R2: the ten weighted densities, shape [10, nz, ny, nx]."""
        if rho_hat is None:
            rho_hat = dft(rho)
        acc = [0.0] * fmt.NALPHA
        for i in range(self.S):
            w = self.w[i]
            acc[0] = acc[0] + rho_hat[i] * w["w0"]
            acc[1] = acc[1] + rho_hat[i] * w["w1"]
            acc[2] = acc[2] + rho_hat[i] * w["w2"]
            acc[3] = acc[3] + rho_hat[i] * w["w3"]
            for d in range(3):
                acc[4 + d] = acc[4 + d] + rho_hat[i] * w["wv1"][d]
                acc[7 + d] = acc[7 + d] + rho_hat[i] * w["wv2"][d]
        return np.stack([_real(a * np.ones(self.shape), f"n[{a_i}]", check)
                         for a_i, a in enumerate(acc)])

    def back_convolution(self, dphi, check=True):
        """R4: c_HS per species from the ten derivative fields."""
        dh = dft(dphi)
        c = np.empty((self.S,) + self.shape)
        for i in range(self.S):
            w = self.w[i]
            acc = (dh[0] * w["w0"] + dh[1] * w["w1"] + dh[2] * w["w2"] + dh[3] * w["w3"])
            for d in range(3):
                acc = acc + dh[4 + d] * np.conj(w["wv1"][d]) + dh[7 + d] * np.conj(w["wv2"][d])
            c[i] = -_real(acc, f"c_hs[{i}]", check)
        return c

    def potential_hat(self, rho_hat):
        """R5: Fourier image of beta e phi (zero mode set to 0)."""
        src = np.zeros(self.shape, complex)
        for j in range(self.S):
            src = src + self.z[j] * rho_hat[j]
        if self.qhat is not None:
            src = src + self.qhat
        with np.errstate(divide="ignore", invalid="ignore"):
            out = 4.0 * math.pi * self.lB * src / self.D
        out[0, 0, 0] = 0.0
        return out

    def potential(self, rho, check=True):
        """beta e phi in real space."""
        if not self.es:
            return np.zeros(self.shape)
        return _real(self.potential_hat(dft(rho)), "phi", check)

    def screening(self, rho_hat, check=True):
        """R6: c_SC per species (bulk-fluid expansion around the bath)."""
        c = np.empty((self.S,) + self.shape)
        for i in range(self.S):
            acc = np.zeros(self.shape, complex)
            for j in range(self.S):
                d = rho_hat[j].copy()
                d[0, 0, 0] -= self.N * self.rho_b[j]
                acc = acc + self.Chat[i][j] * d
            c[i] = _real(acc, f"c_sc[{i}]", check)
        return c

    def evaluate(self, rho, check=True):
        """Full residual evaluation; returns a dict with every intermediate and G."""
        rho = np.asarray(rho, float)
        rho_hat = dft(rho)
        n = self.weighted_densities(rho, rho_hat, check)
        d = fmt.dphi(n, self.functional)
        c_hs = self.back_convolution(d, check)
        E = c_hs.copy()
        phi = np.zeros(self.shape)
        c_sc = np.zeros_like(c_hs)
        if self.es:
            phi = _real(self.potential_hat(rho_hat), "phi", check)
            c_sc = self.screening(rho_hat, check)
            for i in range(self.S):
                E[i] = E[i] + c_sc[i] - self.z[i] * phi
        G = np.zeros_like(rho)
        for i in range(self.S):
            expo = self.mu_hs[i] - self.vext[i] + E[i]
            G[i] = np.where(self.mask[i], self.rho_b[i] * np.exp(np.where(self.mask[i], expo, 0.0)), 0.0)
        n3max = float(np.max(n[3])) if np.all(np.isfinite(n[3])) else math.inf
        return {"rho_hat": rho_hat, "n": n, "dphi": d, "c_hs": c_hs, "phi": phi, "c_sc": c_sc,
                "E": E, "G": G, "n3max": n3max}

    def G(self, rho):
        return self.evaluate(rho)["G"]

    # ------------------------------------------------------------------ norms
    def sqnorm(self, u):
        """Squared weighted L2 norm over fluid nodes: sum_i sum_fluid (u_i / rho_b_i)^2."""
        tot = 0.0
        with np.errstate(over="ignore", invalid="ignore"):
            for i in range(self.S):
                tot += float(np.sum(np.where(self.mask[i], u[i] / self.rho_b[i], 0.0) ** 2))
        return tot if math.isfinite(tot) else math.inf   # a non-finite trial point is never accepted

    def residual_norm(self, sq):
        """r = sqrt(f / number of fluid nodes over all species)."""
        return math.sqrt(sq / max(self.nfluid, 1))

    def free_energy_hs(self, rho):
        """F_HS = h^3 sum_x Phi(n(x)) (kT units), used to pin c_HS as its gradient."""
        n = self.weighted_densities(rho)
        return float(np.prod(self.h) * np.sum(fmt.phi(n, self.functional)))
