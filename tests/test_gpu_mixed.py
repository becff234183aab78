"""GPU: FP32-mixed precision and the graph-launched step runner, against the FP64 oracle.

FP32-mixed targets: the solve reaches the requested residual as measured by an FP64
evaluation, and the density agrees with the FP64 oracle's to 1e-5 relative.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import picard, residual
from paper_0910_1531_amd import _abi

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solver(prob, precision):
    from paper_0910_1531_amd.solver import from_problem
    return from_problem(prob, precision=precision)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


@pytest.mark.parametrize("case", ["sphere", "pore", "wall"])
def test_mixed_solve_reaches_tolerance_and_matches_oracle(case):
    if case == "sphere":
        p, tol = W.charged_sphere(n=32, h=0.1), 1e-8
    elif case == "pore":
        p, tol = W.charged_pore(n=48, h=0.05), 1e-8
    else:
        p, tol = W.config_hs_wall(), 1e-10
    _say(f"mixed solve {case} {p.n}")
    st = residual.Setup(p)
    ref = picard.solve(st, p.initial_density(), 1e-12)
    sol = _solver(p, _abi.DFT_FP32_MIXED)
    x = _dev(p.initial_density())
    it, r, status = sol.solve(x, tol, 2000)
    stats = sol.stats()
    err = _rel(x.cpu().numpy(), ref.rho)
    _say(f"  iters={it} r={r:.3e} refresh={stats['fp64_refresh']} rho_err={err:.2e} oracle_iters={ref.iters}")
    assert status == 0 and r <= tol
    assert stats["fp64_refresh"] >= 2
    assert err < 1e-5
    # an independent FP64 evaluation of the returned density confirms the residual
    sol64 = _solver(p, _abi.DFT_FP64)
    _, r64 = sol64.residual(x)
    assert r64 <= tol * 1.0001
    rr = st.residual_norm(st.sqnorm(x.cpu().numpy() - st.G(x.cpu().numpy())))
    assert rr == pytest.approx(r64, rel=1e-6)


def test_mixed_residual_at_reference_is_the_fp64_residual():
    p = W.charged_sphere(n=32, h=0.1)
    rho = _dev(W.random_density(p, seed=4, amplitude=0.2))
    m = _solver(p, _abi.DFT_FP32_MIXED)
    d = _solver(p, _abi.DFT_FP64)
    m.set_reference(rho)
    Gm, rm = m.residual(rho)
    Gd, rd = d.residual(rho)
    assert _rel(Gm.cpu().numpy(), Gd.cpu().numpy()) < 1e-14
    assert rm == pytest.approx(rd, rel=1e-12)
    # a nearby density: FP32 error proportional to the distance from the reference
    rho2 = rho * (1 + 1e-3 * torch.sin(torch.arange(rho.numel(), device="cuda", dtype=torch.float64)).reshape(rho.shape))
    Gm2, _ = m.residual(rho2)
    Gd2, _ = d.residual(rho2)
    e = _rel(Gm2.cpu().numpy(), Gd2.cpu().numpy())
    _say(f"mixed vs fp64 G at 1e-3 from the reference: {e:.2e}")
    assert e < 1e-8


@pytest.mark.parametrize("n", [64, 96])
def test_mixed_difference_is_finite_where_the_densities_vanish(n):
    """The pore excludes most of the box, so n2 and nV2 vanish there and only FP32 noise of
    the transforms remains; the nodewise FP32 difference of dPhi must stay finite (a product of
    two floored n2^2 underflows) and close to the FP64 evaluation."""
    p = W.charged_pore(n=n, h=0.025 * 256 / n)
    d = _solver(p, _abi.DFT_FP64)
    m = _solver(p, _abi.DFT_FP32_MIXED)
    rho = _dev(p.initial_density())
    d.solve(rho, 1e-6, 200, raise_on_fail=False)
    m.set_reference(rho)
    g = torch.Generator(device="cuda").manual_seed(7)
    for k in range(4):
        pert = rho * (1 + 1e-3 * (2 * torch.rand(rho.shape, generator=g, device="cuda", dtype=torch.float64) - 1))
        Gm, rm = m.residual(pert)
        Gd, rd = d.residual(pert)
        e = _rel(Gm.cpu().numpy(), Gd.cpu().numpy())
        _say(f"  pore{n} perturbation {k}: r mixed {rm:.6e} fp64 {rd:.6e}, G rel diff {e:.1e}")
        assert np.isfinite(rm) and torch.isfinite(Gm).all()
        assert rm == pytest.approx(rd, rel=1e-4)
        assert e < 1e-6


def test_run_equals_repeated_steps():
    p = W.charged_sphere(n=32, h=0.1)
    _say("dft_run vs dft_picard_step")
    a = _solver(p, _abi.DFT_FP64)
    b = _solver(p, _abi.DFT_FP64)
    xa = _dev(p.initial_density())
    xb = xa.clone()
    for _ in range(5):
        a.picard_step(xa)
    acc, r = b.run(xb, 5)
    assert acc == 5
    assert torch.equal(xa, xb)
    # continuing the run keeps the state
    acc2, r2 = b.run(xb, 3)
    for _ in range(3):
        a.picard_step(xa)
    assert torch.equal(xa, xb) and r2 < r


@pytest.mark.parametrize("n", [(64, 3, 3), (32, 1, 9), (12, 3, 9), (256, 1, 3)])
def test_mixed_residual_with_an_odd_row_count(n):
    # An odd number of x rows (n_y n_z) leaves the last row pair of the x passes half empty.
    # Wave-private (64, 256), other compiled (32) and run-time (12) x lengths, and grids with
    # n_y = 1: the FP32-mixed residual near its reference against the FP64 one (1e-6), and the
    # FP64 one against the oracle (1e-11 of the maximum: the perturbation below is rough at the
    # grid scale; a wrong half-empty pair would be off by far more).
    from test_gpu_parity import mixture
    p = mixture(n, S=2, es=True)
    rho = W.random_density(p, seed=11, amplitude=0.3)
    st = residual.Setup(p)
    d = _solver(p, _abi.DFT_FP64)
    m = _solver(p, _abi.DFT_FP32_MIXED)
    x = _dev(rho)
    m.set_reference(x)
    x2 = x * (1 + 0.05 * torch.sin(torch.arange(x.numel(), device="cuda", dtype=torch.float64)).reshape(x.shape))
    Gm, rm = m.residual(x2)
    Gd, rd = d.residual(x2)
    ref = st.evaluate(x2.cpu().numpy())
    em = _rel(Gm.cpu().numpy(), Gd.cpu().numpy())
    ed = _rel(Gd.cpu().numpy(), ref["G"])
    _say(f"odd rows n={n}: FP32-mixed vs FP64 {em:.1e}, FP64 vs oracle {ed:.1e}")
    assert ed < 1e-11
    assert em < 1e-6
