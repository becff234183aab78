"""Newton-Krylov solve of the Euler-Lagrange fixed point (dft_newton) on the GPU.

The fixed point rho = G(rho) is the plain definition both solvers must reach: the Newton
result is compared with the oracle's Picard solution where that converges, and otherwise
(dense hard spheres at packing 0.4, where the Picard line search stalls) checked by the
oracle's own residual evaluation at the GPU's density.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import picard, residual
from paper_0910_1531_amd import _abi
from paper_0910_1531_amd.solver import from_problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


@pytest.mark.parametrize("case", ["sphere32", "pore48", "wall_c1"])
def test_newton_reaches_the_oracle_fixed_point(case):
    if case == "sphere32":
        p = W.charged_sphere(n=32, h=0.1)
    elif case == "pore48":
        p = W.charged_pore(n=48, h=0.0625)
    else:
        p = W.config_hs_wall()
    st = residual.Setup(p)
    ref = picard.solve(st, p.initial_density(), 1e-12, max_iter=3000)
    sol = from_problem(p)
    x = _dev(p.initial_density())
    it, cg, r, status = sol.newton(x, 1e-11, 60)
    err = _rel(x.cpu().numpy(), ref.rho)
    _say(f"  {case}: Newton {it} steps, {cg} CG iterations, r {r:.1e}; oracle Picard {ref.iters} iterations; "
         f"rho rel diff {err:.1e}")
    assert status == 0 and r <= 1e-11
    assert err < 1e-9
    assert it < ref.iters


def test_newton_converges_where_picard_stalls():
    """Hard spheres at packing 0.4 against a wall (h = sigma / 32): the Picard line search
    stalls (oracle and GPU alike).  Newton-Krylov reaches the fixed point by continuation in
    the bath density (each solution, rescaled, starts the next packing), and the oracle's own
    residual at the GPU's density confirms it."""
    x = None
    prev = None
    for eta in (0.3, 0.35, 0.4):
        p = W.hs_wall_nm(eta, n=(384, 1, 1))
        sol = from_problem(p)
        if x is None:
            x = _dev(p.initial_density())
        else:
            x = x * (p.rho_bulk[0] / prev.rho_bulk[0])
        it, cg, r, status = sol.newton(x, 1e-10, 100)
        _say(f"  packing {eta}: Newton {it} steps, {cg} CG iterations, r {r:.1e}, status {status}")
        assert status == 0 and r <= 1e-10
        prev = p
    st = residual.Setup(p)
    rho = x.cpu().numpy()
    r_oracle = st.residual_norm(st.sqnorm(rho - st.G(rho)))
    m = int(round(p.radius[0] / p.h[0]))
    _say(f"  oracle residual at the GPU density {r_oracle:.1e}; contact/betaP - 1 = {rho[0, 0, 0, m] / st.betaP - 1:.3e}")
    assert r_oracle <= 1e-9
