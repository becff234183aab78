"""GPU parity of the alternative hard-sphere functionals against the oracle: Rosenfeld's
original vector form (Percus-Yevick bath) and White Bear (BMCSL bath), selected through
dft_params.hs_functional.

Bars as for eq. (Phi): FP64 operators to 1e-12 of each field's maximum, converged densities
to 1e-9 relative; FP32-mixed solves to 1e-5 relative (the mixed path's bar).  The dense wall
cases put n3 on both sides of 0.1, where the White Bear factor switches from its Taylor series
to its closed form.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as oadj
from oracle import bulk as obulk
from oracle import picard, residual
from paper_0910_1531_amd import _abi
from paper_0910_1531_amd.solver import from_problem
from test_gpu_parity import mixture

pytestmark = pytest.mark.gpu

FUNCTIONALS = ["rosenfeld", "whitebear"]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _problem(case, functional):
    if case == "wall":
        p = W.config_hs_wall()
    elif case == "mix12":
        p = mixture((12, 6, 9), S=2)            # run-time-length kernels
    elif case == "mix32":
        p = mixture((32, 32, 32), S=2)          # compiled-length kernels
    else:
        p = mixture((96, 64, 48), S=3)
    p.hs_functional = functional
    return p


@pytest.mark.parametrize("functional", FUNCTIONALS)
@pytest.mark.parametrize("case", ["wall", "mix12", "mix32", "mix96"])
def test_operators_match_oracle(case, functional):
    p = _problem(case, functional)
    _say(f"operators {case} {functional}")
    st = residual.Setup(p)
    rho = W.random_density(p, seed=5, amplitude=0.4)
    ref = st.evaluate(rho)
    if case == "wall":
        n3 = ref["n"][3]
        assert n3.min() < 0.1 < n3.max()
    sol = from_problem(p)
    out = sol.operators(_dev(rho))
    torch.cuda.synchronize()
    errs = {}
    for a in range(10):
        errs[f"dphi{a}"] = _rel(out["dphi"][a].cpu().numpy(), ref["dphi"][a])
    errs["E"] = _rel(out["c"].cpu().numpy(), ref["E"])
    G, r = sol.residual(_dev(rho))
    errs["G"] = _rel(G.cpu().numpy(), ref["G"])
    _say("  max rel errors: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v < 1e-12}
    assert not bad, bad
    assert r == pytest.approx(st.residual_norm(st.sqnorm(rho - ref["G"])), rel=1e-12)


@pytest.mark.parametrize("functional", FUNCTIONALS)
def test_uniform_bath_is_a_fixed_point(functional):
    # Without the wall the bath must reproduce itself: the host's closed-form bath chemical
    # potential equals the functional's own bulk derivative on the device.
    p = W.config_hs_wall()
    p.beta_vext = None
    p.hs_functional = functional
    sol = from_problem(p)
    rb = p.initial_density()
    G, r = sol.residual(_dev(rb))
    _say(f"bath {functional}: r = {r:.1e}")
    assert _rel(G.cpu().numpy(), rb) < 1e-14
    assert r < 1e-14


@pytest.mark.parametrize("precision", [_abi.DFT_FP64, _abi.DFT_FP32_MIXED])
@pytest.mark.parametrize("functional", FUNCTIONALS)
def test_solve_matches_oracle(functional, precision):
    p = W.config_hs_wall()
    p.hs_functional = functional
    st = residual.Setup(p)
    ref = picard.solve(st, p.initial_density(), 1e-11, max_iter=3000)
    sol = from_problem(p, precision=precision)
    x = _dev(p.initial_density())
    it, r, status = sol.solve(x, 1e-10, 3000)
    err = _rel(x.cpu().numpy(), ref.rho)
    _say(f"solve {functional} precision {precision}: {it} iterations (oracle {ref.iters}), r {r:.1e}, "
         f"rho rel diff {err:.1e}")
    assert status == 0 and r <= 1e-10
    assert err < (1e-9 if precision == _abi.DFT_FP64 else 1e-5)


def test_white_bear_wall_contact_and_1d_oracle():
    # Packing 0.3 against a hard wall on the cells of the hard-sphere accuracy study: the 3-D
    # solution equals the oracle's 1-D solution of the same discrete problem, and the contact
    # density approaches the Carnahan-Starling pressure (the White Bear bulk) up to the grid's
    # first-order error.
    eta = 0.3
    p = W.hs_wall_nm(eta)
    p.hs_functional = "whitebear"
    sol = from_problem(p)
    x = _dev(p.initial_density())
    it, r, st = sol.solve(x, 1e-10, 3000)
    assert st == 0 and r <= 1e-10
    rho = x.cpu().numpy()[0]
    spread = np.max(np.abs(rho - rho[:1, :1, :])) / np.max(rho)
    q = W.hs_wall_nm(eta, n=(p.n[0], 1, 1))
    q.hs_functional = "whitebear"
    s1 = picard.solve(residual.Setup(q), q.initial_density(), 1e-11, max_iter=3000)
    ref = s1.rho[0, 0, 0, :]
    dev = np.max(np.abs(rho[0, 0, :] - ref)) / np.max(ref)
    m = int(round(p.radius[0] / p.h[0]))
    rho_b = q.rho_bulk[0]
    betaP_cs = rho_b * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
    assert betaP_cs == pytest.approx(obulk.bmcsl_pressure(q.rho_bulk, 2 * q.radius), rel=1e-12)
    err = rho[0, 0, m] / betaP_cs - 1.0
    _say(f"White Bear wall eta {eta}: {it} iterations, contact/betaP_CS - 1 = {err:.3e}, "
         f"spread {spread:.1e}, vs 1-D oracle {dev:.1e}")
    assert spread <= 1e-12
    assert dev <= 1e-8
    assert abs(err) < 0.1


@pytest.mark.parametrize("functional", FUNCTIONALS)
def test_newton_reaches_the_oracle_fixed_point(functional):
    p = W.config_hs_wall()
    p.hs_functional = functional
    ref = picard.solve(residual.Setup(p), p.initial_density(), 1e-12, max_iter=3000)
    sol = from_problem(p)
    x = _dev(p.initial_density())
    it, cg, r, status = sol.newton(x, 1e-11, 60)
    err = _rel(x.cpu().numpy(), ref.rho)
    _say(f"Newton {functional}: {it} steps, {cg} CG iterations, r {r:.1e}; oracle Picard {ref.iters}; "
         f"rho rel diff {err:.1e}")
    assert status == 0 and r <= 1e-11
    assert err < 1e-9


def test_white_bear_adjoint_matches_oracle():
    p = W.charged_sphere(n=16, h=0.1, sigma=(0.3, 0.24), conc=(0.5, 0.5), sphere_radius=0.25,
                         sphere_charge=-1.0)
    p.hs_functional = "whitebear"
    d = W._dist_to_point(p.n, p.h, p.extra["centre"])
    mask = (d >= 0.39) & (d < 0.55)
    st = residual.Setup(p)
    rho = picard.solve(st, p.initial_density(), 1e-13).rho
    g = np.zeros_like(rho)
    g[0][mask] = np.prod(p.h)
    ref = oadj.gradient(p, rho, g)
    sol = from_problem(p)
    out = sol.adjoint(_dev(rho), _dev(g), tol=1e-12)
    _say(f"White Bear adjoint: CG iterations {out['iters']}, residual {out['resid']:.1e}")
    for name, got, want in [("vext", out["vext"].cpu().numpy(), ref["vext"]),
                            ("rho_bulk", out["rho_bulk"], ref["rho_bulk"]),
                            ("sigma", out["sigma"], ref["sigma"])]:
        got, want = np.asarray(got, float).ravel(), np.asarray(want, float).ravel()
        scale = np.abs(want).max()
        dev = np.abs(got - want)
        _say(f"  {name}: max rel dev {dev.max() / scale:.2e}")
        assert np.all(dev <= 1e-5 * np.maximum(np.abs(want), 1e-3 * scale)), name
