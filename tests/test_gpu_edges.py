"""Degenerate inputs and error paths on the GPU: no fluid node, max_iter reached, a non-finite
density, over-packed densities, and the largest number of species (eight, run-time-length z
kernels) against the oracle."""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import residual
from paper_0910_1531_amd import _abi
from paper_0910_1531_amd.solver import from_problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_every_centre_excluded_is_an_argument_error():
    p = W.hard_wall(n=(16, 8, 8), h=0.2, sigma=1.0, eta=0.2)
    p.beta_vext = np.full((1,) + p.shape, np.inf)
    with pytest.raises(_abi.DftError) as ei:
        from_problem(p)
    assert ei.value.status == 1                      # DFT_E_INVALID_ARG
    _say(f"  no fluid node: {ei.value}")


@pytest.mark.parametrize("precision", [_abi.DFT_FP64, _abi.DFT_FP32_MIXED])
def test_max_iter_reached_reports_not_converged(precision):
    p = W.config_hs_wall()
    sol = from_problem(p, precision=precision)
    x = _dev(p.initial_density())
    it, r, st = sol.solve(x, 1e-12, 3, raise_on_fail=False)
    assert st == 7 and it == 3 and math.isfinite(r) and r > 1e-12
    assert torch.isfinite(x).all()


def test_non_finite_and_overpacked_densities_give_an_infinite_residual():
    p = W.config_hs_wall()
    sol = from_problem(p)
    rho = p.initial_density()
    bad = rho.copy()
    bad[0, 3, 4, 20] = np.nan
    G, r = sol.residual(_dev(bad))
    assert r == math.inf
    dense = rho * 6.0                              # packing 1.2 in the bulk: n3 >= 1 there
    G, r = sol.residual(_dev(dense))
    assert r == math.inf
    G, r = sol.residual(_dev(rho))                  # and the ctx still evaluates normally
    st = residual.Setup(p)
    ref = st.evaluate(rho)["G"]
    assert float(np.max(np.abs(G.cpu().numpy() - ref)) / np.max(np.abs(ref))) < 1e-12


@pytest.mark.parametrize("n", [(12, 8, 9), (16, 16, 16)])
def test_eight_species_match_the_oracle(n):
    # DFT_MAX_SPECIES species, neutral, charged: the electrostatic z kernels of the compiled
    # lengths take at most four species, so these run on the run-time-length kernels.
    S = _abi.MAX_SPECIES
    R = np.linspace(0.08, 0.2, S)
    z = np.array([1.0, -1.0, 2.0, -2.0, 1.0, -1.0, 3.0, -3.0])[:S]
    rho = np.full(S, 0.4)
    p = W.Problem(name="eight", n=n, h=(0.09, 0.1, 0.11), radius=R, valence=z, rho_bulk=rho, bjerrum=0.3,
                  electrostatics=True)
    d = W._dist_to_point(p.n, p.h, (0.4, 0.3, 0.5))
    bv = np.zeros((S,) + p.shape)
    for k in range(S):
        bv[k][d < 0.1 + R[k]] = np.inf
    p.beta_vext = bv
    st = residual.Setup(p)
    x = W.random_density(p, seed=11, amplitude=0.3)
    ref = st.evaluate(x)
    sol = from_problem(p)
    G, r = sol.residual(_dev(x))
    err = float(np.max(np.abs(G.cpu().numpy() - ref["G"])) / np.max(np.abs(ref["G"])))
    _say(f"  eight species {n}: G rel err {err:.1e}")
    assert err < 1e-12
    assert r == pytest.approx(st.residual_norm(st.sqnorm(x - ref["G"])), rel=1e-12)
