"""torch.autograd around the fixed point of the Euler-Lagrange equation (eq. rhoEquation).

forward:  rho* = solution of rho = G(rho; beta V, sigma, rho_bulk)      (dft_setup + dft_solve)
backward: the implicit adjoint at rho* (dft_adjoint): for an upstream gradient g = dO/drho*,
          dO/d(beta V_k(x)) = -w_k(x), and dO/d sigma_k, dO/d rho_bulk_k from the spectral and
          bath sums of the library, with w solving (diag(G)^-1 - H) w = g on fluid nodes.

Marshalling only: the solve and the adjoint run in the HIP library.  Hard-core exclusion
(beta V = +inf) is held fixed, as the adjoint assumes; the gradient there is 0.
"""
import dataclasses

import torch

from . import _abi
from .solver import Solver, make_params


@dataclasses.dataclass
class FixedPointConfig:
    """Everything of the problem that is not differentiated (dft_params fields, solver controls)."""
    n: tuple
    h: tuple
    valence: tuple
    bjerrum: float = 0.0
    electrostatics: bool = False
    fixed_charge: object = None          # device [nz][ny][nx] float64 or None
    precision: int = _abi.DFT_FP64
    flags: int = 0
    hs_functional: str = "rslt"
    eta_cap: float = 0.0
    tol: float = 1e-10
    max_iter: int = 5000
    adjoint_tol: float = 1e-11
    adjoint_max_iter: int = 1000


class FixedPointDensity(torch.autograd.Function):
    """rho* (device [S][nz][ny][nx] float64) as a function of beta V (device, same shape),
    sigma [S] and rho_bulk [S] (float64 tensors on any device)."""

    @staticmethod
    def forward(ctx, beta_vext, sigma, rho_bulk, cfg, rho0):
        S = len(cfg.valence)
        if beta_vext.dtype != torch.float64 or beta_vext.device.type != "cuda":
            raise ValueError("beta_vext must be a float64 CUDA tensor")
        radius = [0.5 * float(s) for s in sigma.detach().cpu().tolist()]
        rb = [float(v) for v in rho_bulk.detach().cpu().tolist()]
        if len(radius) != S or len(rb) != S:
            raise ValueError("sigma and rho_bulk need one entry per species")
        params = make_params(cfg.n, cfg.h, radius, cfg.valence, rb, cfg.bjerrum, cfg.electrostatics,
                             cfg.precision, cfg.eta_cap, cfg.flags, cfg.hs_functional)
        sol = Solver(params, beta_vext.detach().contiguous(), cfg.fixed_charge, device=beta_vext.device)
        if rho0 is None:
            rho = torch.zeros(sol.shape, dtype=torch.float64, device=beta_vext.device)
            for k in range(S):
                rho[k] = torch.where(torch.isfinite(beta_vext[k]), rb[k], 0.0)
        else:
            rho = rho0.detach().clone().contiguous()
        sol.solve(rho, cfg.tol, cfg.max_iter)
        ctx.sol = sol
        ctx.cfg = cfg
        ctx.sigma_meta = (sigma.dtype, sigma.device)
        ctx.rb_meta = (rho_bulk.dtype, rho_bulk.device)
        ctx.save_for_backward(rho)
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        (rho,) = ctx.saved_tensors
        sol, cfg = ctx.sol, ctx.cfg
        g = grad_rho.detach().to(torch.float64).contiguous()
        out = sol.adjoint(rho, g, tol=cfg.adjoint_tol, max_iter=cfg.adjoint_max_iter,
                          vext=ctx.needs_input_grad[0])
        d_vext = out["vext"] if ctx.needs_input_grad[0] else None
        d_sigma = torch.tensor(out["sigma"], dtype=ctx.sigma_meta[0], device=ctx.sigma_meta[1]) \
            if ctx.needs_input_grad[1] else None
        d_rb = torch.tensor(out["rho_bulk"], dtype=ctx.rb_meta[0], device=ctx.rb_meta[1]) \
            if ctx.needs_input_grad[2] else None
        return d_vext, d_sigma, d_rb, None, None


def fixed_point_density(beta_vext, sigma, rho_bulk, cfg: FixedPointConfig, rho0=None):
    """rho* with gradients to beta V, sigma (diameters) and rho_bulk through the implicit adjoint."""
    return FixedPointDensity.apply(beta_vext, sigma, rho_bulk, cfg, rho0)
