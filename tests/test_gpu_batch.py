"""GPU batches: many state points solved together equal the same points solved one by one,
and the batched electrolyte workload converges in FP32-mixed."""
import sys
import time

import numpy as np
import pytest
import torch

import workloads as W
from paper_0910_1531_amd import _abi

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision", [_abi.DFT_FP64, _abi.DFT_FP32_MIXED])
def test_batch_equals_individual_solves(precision):
    from paper_0910_1531_amd.solver import Batch, from_problem
    pts = W.batch_points(count=7, seed=4, h=0.1, sizes=(16, 24, 32))
    _say(f"batch of {len(pts)} points, sizes {[p.n[0] for p in pts]}, precision {precision}")
    b = Batch(pts, precision=precision)
    rhos = [_dev(p.initial_density()) for p in pts]
    its, norms, sts = b.solve(rhos, 1e-9, 500)
    assert all(s == 0 for s in sts) and all(r <= 1e-9 for r in norms)
    for i, p in enumerate(pts):
        sol = from_problem(p, precision=precision)
        x = _dev(p.initial_density())
        it, r, st = sol.solve(x, 1e-9, 500)
        assert st == 0 and it == its[i]
        assert torch.equal(x, rhos[i]), i
        assert b.stats(i)["iterations"] == it


def test_batched_electrolyte_workload_fp32_mixed():
    """64 state points (1:1 / 2:1 salts, 0.01-1 M, sigma 0.2-0.4 nm, charged spheres) on
    64^3 / 96^3 / 128^3 grids, FP32-mixed, to residual 1e-8."""
    from paper_0910_1531_amd.solver import Batch
    pts = W.batch_points(count=64, seed=4)
    sizes = [p.n[0] for p in pts]
    _say(f"64-point batch: {sizes.count(64)} x 64^3, {sizes.count(96)} x 96^3, {sizes.count(128)} x 128^3")
    b = Batch(pts, precision=_abi.DFT_FP32_MIXED)
    rhos = [_dev(p.initial_density()) for p in pts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, norms, sts = b.solve(rhos, 1e-8, 2000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _say(f"  solved in {dt:.2f} s; iterations min/median/max {min(its)}/{int(np.median(its))}/{max(its)}")
    assert all(s == 0 for s in sts), sts
    assert max(norms) <= 1e-8
    # one point of each grid size against the FP64 oracle's converged densities (sampled; written
    # by tests/golden/make_oracle_solutions.py)
    from test_gpu_fullsize import golden
    for N in (64, 96, 128):
        meta, idx, want = golden(f"batch{N}")
        i = [p.name for p in pts].index(meta["problem"])
        assert list(pts[i].n) == meta["grid"]
        got = rhos[i].cpu().numpy().ravel()[idx]
        err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        _say(f"  point {i} ({N}^3): {its[i]} iterations (oracle {meta['iterations']} to 1e-12), "
             f"rho vs oracle {err:.2e}")
        assert err < 1e-5


def test_batch_groups_split_by_functional():
    # Points of one grid that use different hard-sphere functionals form separate groups and each
    # solves exactly as it does alone.
    from paper_0910_1531_amd.solver import Batch, from_problem
    pts = W.batch_points(count=4, seed=6, h=0.1, sizes=(16,))
    for p, fn in zip(pts, ["rslt", "whitebear", "rosenfeld", "whitebear"]):
        p.hs_functional = fn
    b = Batch(pts)
    rhos = [_dev(p.initial_density()) for p in pts]
    its, norms, sts = b.solve(rhos, 1e-9, 500)
    assert all(s == 0 for s in sts) and all(r <= 1e-9 for r in norms)
    for i, p in enumerate(pts):
        sol = from_problem(p)
        x = _dev(p.initial_density())
        it, r, st = sol.solve(x, 1e-9, 500)
        assert st == 0 and it == its[i]
        assert torch.equal(x, rhos[i]), i
