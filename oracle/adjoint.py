"""Implicit-adjoint gradient of an observable through the converged fixed point.

At the solution rho* = G(rho*; theta) of eq. (rhoEquation), an observable O(rho*)
has dO/dtheta = lambda^T dG/dtheta with (I - J^T) lambda = dO/drho, J = dG/drho.
Writing G = rho_b exp(beta mu_b - beta V + E[rho]) on fluid nodes, J = diag(G) H with
H = dE/drho (symmetric: every convolution is paired with its transpose and Phi'' is a
Hessian), so w = G o lambda solves (diag(G)^-1 - H) w = dO/drho on fluid nodes
(w = 0 elsewhere).  That matrix is the Hessian of the grand potential, symmetric
positive definite at a stable solution, so conjugate gradients apply.

This module is the oracle's own construction, independent of the GPU path:
  * H u is a central difference of the exponent E along u (step 1e-5 relative);
  * the linear system is solved with scipy's conjugate-gradient routine,
    preconditioned by diag(G);
  * parameter derivatives of G at fixed rho* (and fixed hard-core masks) are central
    differences of ln G from setups rebuilt with the perturbed parameter.
Gradients: d/d(beta V_k(x)) = -w_k(x); d/d rho_b,k and d/d sigma_k = sum_i sum_x
w_i d ln G_i / d theta.

Pins: tests/test_oracle_adjoint.py compares these gradients with central differences of
O through complete re-solves of the fixed point.
"""
import copy

import numpy as np
from scipy.sparse.linalg import LinearOperator, cg

from . import residual


def _exponent(st, rho):
    return st.evaluate(rho, check=False)["E"]


def hessian_vec(st, rho, u, rel=1e-5):
    """H u = dE/drho . u by a central difference of the exponent."""
    scale = rel * max(np.max(np.abs(rho)), 1e-300) / max(np.max(np.abs(u)), 1e-300)
    return (_exponent(st, rho + scale * u) - _exponent(st, rho - scale * u)) / (2.0 * scale)


def adjoint_weights(st, rho, dO_drho, tol=1e-12, maxiter=500):
    """w = G o lambda on fluid nodes, solving (1/G - H) w = dO/drho by preconditioned CG."""
    G = st.evaluate(rho)["G"]
    fluid = st.mask & (G > 0)
    shape = rho.shape
    idx = np.flatnonzero(fluid)
    Gf = G.ravel()[idx]

    def embed(v):
        full = np.zeros(rho.size)
        full[idx] = v
        return full.reshape(shape)

    def matvec(v):
        return v / Gf - hessian_vec(st, rho, embed(v)).ravel()[idx]

    A = LinearOperator((idx.size, idx.size), matvec=matvec, dtype=float)
    M = LinearOperator((idx.size, idx.size), matvec=lambda v: Gf * v, dtype=float)
    b = np.asarray(dO_drho, float).ravel()[idx]
    w, info = cg(A, b, x0=Gf * b, rtol=tol, atol=0.0, maxiter=maxiter, M=M)
    if info != 0:
        raise RuntimeError(f"adjoint CG did not converge (info={info})")
    return embed(w), G


def _perturbed(prob, field, k, delta):
    p = copy.deepcopy(prob)
    if field == "rho_bulk":
        p.rho_bulk = np.array(p.rho_bulk, float)
        p.rho_bulk[k] += delta
    elif field == "sigma":
        p.radius = np.array(p.radius, float)
        p.radius[k] += 0.5 * delta
    else:
        raise ValueError(field)
    return p


def dlnG_dtheta(prob, rho, field, k, rel=1e-6, cutoff="contact"):
    """Central difference of ln G_i(rho) (fluid nodes) in rho_bulk[k] or sigma[k], rho fixed."""
    base = prob.rho_bulk[k] if field == "rho_bulk" else 2.0 * prob.radius[k]
    d = rel * base
    Gp = residual.Setup(_perturbed(prob, field, k, d), cutoff=cutoff).evaluate(rho)["G"]
    Gm = residual.Setup(_perturbed(prob, field, k, -d), cutoff=cutoff).evaluate(rho)["G"]
    with np.errstate(divide="ignore", invalid="ignore"):
        out = (np.log(Gp) - np.log(Gm)) / (2.0 * d)
    return np.where(np.isfinite(out), out, 0.0)


def gradient(prob, rho, dO_drho, tol=1e-12, cutoff="contact"):
    """dO/d(beta V) [S, ...], dO/d rho_bulk [S] and dO/d sigma [S] at the fixed point rho
    (cutoff: the screening-kernel cutoff of residual.Setup)."""
    st = residual.Setup(prob, cutoff=cutoff)
    w, G = adjoint_weights(st, rho, dO_drho, tol=tol)
    S = prob.nspecies
    d_rho_b = np.array([np.sum(w * dlnG_dtheta(prob, rho, "rho_bulk", k, cutoff=cutoff)) for k in range(S)])
    d_sigma = np.array([np.sum(w * dlnG_dtheta(prob, rho, "sigma", k, cutoff=cutoff)) for k in range(S)])
    return {"vext": -w, "rho_bulk": d_rho_b, "sigma": d_sigma, "w": w}
