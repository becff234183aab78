"""GPU parity on the transform lengths and sizes the configurations run, against the FP64 oracle.

* Grids whose y and z axes take the compiled transform lengths 96 .. 384 (the kernels of the 256^3
  pore, the 128^3 sphere, the 192^3 differentiation workload), with x either a compiled length
  (compact vector layout) or a run-time length (ten-spectrum layout): every operator element by
  element at 1e-12 in FP64, and G of the FP32-mixed evaluation 5 % away from its reference within
  1e-6 of the oracle's G.
* The 256^3 charged pore itself: one FP64 evaluation against the oracle's, element by element, the
  FP32-mixed evaluation near its reference, and the converged FP64 and FP32-mixed solves (the FP64
  solution is a fixed point of the oracle's map to 1e-11; FP32-mixed within 1e-5 of it).
* The 128^3 charged sphere solved to 1e-12: the GPU's densities against the oracle's converged
  densities (sampled, tests/golden/oracle_solutions.npz, written by make_oracle_solutions.py) to
  1e-10 with the same iteration count; FP32-mixed to 1e-8 within 1e-5.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import residual
from paper_0910_1531_amd import _abi
from paper_0910_1531_amd.solver import from_problem

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def golden(name):
    meta = json.load(open(os.path.join(GOLDEN, "oracle_solutions.json")))[name]
    with np.load(os.path.join(GOLDEN, "oracle_solutions.npz"), allow_pickle=False) as f:
        return meta, f[f"{name}_idx"], f[f"{name}_rho"]


def _mixture(n, S):
    from test_gpu_parity import mixture
    return mixture(n, S=S, es=True)


def _perturbed(x):
    ramp = torch.sin(torch.arange(x.numel(), device="cuda", dtype=torch.float64)).reshape(x.shape)
    return x * (1 + 0.05 * ramp)


def _compare_operators(sol, st, rho, ref, tag):
    out = sol.operators(_dev(rho))
    errs = {}
    for a in range(10):
        errs[f"n{a}"] = _rel(out["n"][a].cpu().numpy(), ref["n"][a])
        errs[f"dphi{a}"] = _rel(out["dphi"][a].cpu().numpy(), ref["dphi"][a])
    errs["E"] = _rel(out["c"].cpu().numpy(), ref["E"])
    errs["phi"] = _rel(out["phi"].cpu().numpy(), ref["phi"])
    del out
    G, r = sol.residual(_dev(rho))
    errs["G"] = _rel(G.cpu().numpy(), ref["G"])
    worst = max(errs, key=errs.get)
    _say(f"  {tag}: worst {worst} {errs[worst]:.1e}, G {errs['G']:.1e}")
    bad = {k: v for k, v in errs.items() if not v < 1e-12}
    assert not bad, bad
    assert r == pytest.approx(st.residual_norm(st.sqnorm(rho - ref["G"])), rel=1e-12)


# (grid, species, expected vector layout): y and z on compiled lengths, x compiled (compact layout)
# or a run-time length (ten spectra)
COMPILED = [((16, 256, 256), 3, 1), ((12, 256, 256), 3, 0), ((24, 192, 128), 2, 1), ((18, 128, 192), 3, 0),
            ((16, 128, 384), 2, 1), ((32, 96, 96), 3, 1)]


@pytest.mark.parametrize("n,S,compact", COMPILED)
def test_compiled_lengths_match_oracle(n, S, compact):
    p = _mixture(n, S)
    _say(f"compiled lengths n={n} S={S}")
    st = residual.Setup(p)
    rho = W.random_density(p, seed=3, amplitude=0.4)
    ref = st.evaluate(rho)
    sol = from_problem(p)
    assert sol.stats()["compact_layout"] == compact
    _compare_operators(sol, st, rho, ref, "FP64")
    sol.close()
    # FP32-mixed: transforms of the difference from a reference 5 % away
    m = from_problem(p, precision=_abi.DFT_FP32_MIXED)
    assert m.stats()["compact_layout"] == compact
    x = _dev(rho)
    m.set_reference(x)
    x2 = _perturbed(x)
    G2 = st.G(x2.cpu().numpy())
    Gm, _ = m.residual(x2)
    e = _rel(Gm.cpu().numpy(), G2)
    _say(f"  FP32-mixed G 5 % from the reference vs the oracle: {e:.1e}")
    assert e < 1e-6


@pytest.fixture(scope="module")
def pore256():
    return W.config_pore(n=256)


def test_pore256_evaluation_matches_oracle(pore256):
    p = pore256
    _say("pore 256^3: one oracle evaluation")
    st = residual.Setup(p)
    rho = W.random_density(p, seed=3, amplitude=0.4)
    ref = st.evaluate(rho)
    sol = from_problem(p)
    assert sol.stats()["compact_layout"] == 1
    _compare_operators(sol, st, rho, ref, "pore 256^3 FP64")
    sol.close()
    del ref
    m = from_problem(p, precision=_abi.DFT_FP32_MIXED)
    x = _dev(rho)
    m.set_reference(x)
    x2 = _perturbed(x)
    G2 = st.G(x2.cpu().numpy())
    Gm, _ = m.residual(x2)
    e = _rel(Gm.cpu().numpy(), G2)
    _say(f"  pore 256^3 FP32-mixed G 5 % from the reference vs the oracle: {e:.1e}")
    assert e < 1e-6


def test_pore256_solves_fp64_and_mixed(pore256):
    p = pore256
    _say("pore 256^3: FP64 solve to 1e-12, FP32-mixed to 1e-8")
    st = residual.Setup(p)
    d = from_problem(p)
    x = _dev(p.initial_density())
    it, r, s = d.solve(x, 1e-12, 500)
    assert s == 0 and r <= 1e-12
    xr = x.cpu().numpy()
    r_or = st.residual_norm(st.sqnorm(xr - st.G(xr)))
    m = from_problem(p, precision=_abi.DFT_FP32_MIXED)
    y = _dev(p.initial_density())
    itm, rm, sm = m.solve(y, 1e-8, 500)
    assert sm == 0 and rm <= 1e-8
    err = max(_rel(y[k].cpu().numpy(), xr[k]) for k in range(p.nspecies))
    _say(f"  FP64: {it} iterations, r {r:.2e}, oracle residual at the GPU solution {r_or:.2e}; "
         f"FP32-mixed: {itm} iterations, r {rm:.2e}, rho error vs FP64 {err:.2e}")
    assert r_or < 1e-11
    assert err < 1e-5


@pytest.mark.parametrize("precision", [_abi.DFT_FP64, _abi.DFT_FP32_MIXED])
def test_sphere128_solve_matches_oracle_solution(precision):
    meta, idx, want = golden("sphere128")
    p = W.config_sphere_128()
    assert list(p.n) == meta["grid"]
    sol = from_problem(p, precision=precision)
    x = _dev(p.initial_density())
    tol = 1e-12 if precision == _abi.DFT_FP64 else 1e-8
    it, r, s = sol.solve(x, tol, 500)
    assert s == 0 and r <= tol
    got = x.cpu().numpy().ravel()[idx]
    scale = np.max(np.abs(want))
    err = float(np.max(np.abs(got - want)) / scale)
    _say(f"sphere 128^3 precision {precision}: {it} iterations (oracle {meta['iterations']}), r {r:.2e}, "
         f"rho vs oracle at {idx.size} points {err:.2e}")
    if precision == _abi.DFT_FP64:
        assert it == meta["iterations"]
        assert err < 1e-10
    else:
        assert err < 1e-5
