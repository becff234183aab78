"""Launch-shape autotuner of the compiled-length pass kernels.

Every shape of a tunable pass performs the same arithmetic in the same order, so a
residual evaluated under any schedule must equal the default schedule's bit for bit; the
tuned schedule must be a valid one; and a solve with tuning must equal one without.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from paper_0910_1531_amd import _abi
from paper_0910_1531_amd.solver import from_problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# launch shapes of each tunable pass
NSHAPE = {"y": 10, "z_plain": 10, "z_weights": 6, "z_back": 3, "y_fwd2": 10, "y_species": 10}


def _problems():
    yield "pore48", W.charged_pore(n=48, h=0.0625)
    p = W.charged_sphere(n=(64, 32, 96), h=0.05, sigma=(0.3, 0.24), conc=(0.5, 0.5), sphere_radius=0.3)
    yield "sphere64x32x96", p
    # planes of 24 x 5 pencils: the last y and z tiles of 16 or 32 pencils are partial
    p = W.charged_sphere(n=(8, 24, 24), h=0.05, sigma=(0.3, 0.24), conc=(0.5, 0.5), sphere_radius=0.2)
    yield "sphere8x24x24", p


@pytest.mark.parametrize("precision", [_abi.DFT_FP64, _abi.DFT_FP32_MIXED])
def test_every_shape_gives_the_same_residual(precision):
    for name, p in _problems():
        sol = from_problem(p, precision=precision, flags=_abi.FLAG_NO_AUTOTUNE)
        assert all(v == (0, 0) for v in sol.schedule().values())
        rho = torch.tensor(W.random_density(p, seed=1, amplitude=0.3), dtype=torch.float64, device="cuda")
        if precision == _abi.DFT_FP32_MIXED:
            sol.set_reference(torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda"))
        g0, r0 = sol.residual(rho)
        g0 = g0.clone()
        for ps, nv in NSHAPE.items():
            for v in range(1, nv):
                for t in (0, 1):
                    sched = {k: (0, 0) for k in NSHAPE}
                    sched[ps] = (v, 0) if t == 0 else (0, v)
                    sol.set_schedule(sched)
                    g, r = sol.residual(rho)
                    same = torch.equal(g, g0) and r == r0
                    _say(f"  {name} precision {precision} pass {ps} shape {v} ({'FP32' if t else 'FP64'}): "
                         f"{'identical' if same else 'DIFFERENT'}")
                    assert same, (name, ps, v, t)
        with pytest.raises(RuntimeError):
            sol.set_schedule({"z_weights": (6, 0)})
        sol.close()


def test_tuned_solve_equals_untuned():
    p = W.charged_pore(n=48, h=0.0625, tol=1e-8)
    out = []
    for flags in (0, _abi.FLAG_NO_AUTOTUNE):
        sol = from_problem(p, precision=_abi.DFT_FP32_MIXED, flags=flags)
        sched = sol.schedule()
        _say(f"  flags {flags}: schedule {sched}")
        assert set(sched) == set(NSHAPE)
        for ps, v in sched.items():
            assert 0 <= v[0] < NSHAPE[ps] and 0 <= v[1] < NSHAPE[ps]
        rho = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
        it, r, st = sol.solve(rho, 1e-8, 500)
        assert st == 0
        out.append((it, r, rho.clone()))
        sol.close()
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    assert torch.equal(out[0][2], out[1][2])
