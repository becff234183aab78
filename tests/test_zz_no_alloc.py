"""dft_adjoint_noalloc (the adjoint with its workspace in the library's static device array) against
dft_adjoint with a caller workspace, through the C ABI: two calls in a row on one GPU, the second on a
smaller problem, each equal to the workspace entry point's result; an oversized problem is refused."""
import ctypes
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


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _case(name):
    if name == "pore32":
        p = W.charged_pore(n=32, h=0.0625)
        mask = W.pore_observable_mask(p, half_length=0.6)
    else:
        p = W.charged_sphere(n=16, h=0.1, sigma=(0.3, 0.24), conc=(0.5, 0.5), sphere_radius=0.25,
                             sphere_charge=-1.0)
        d = W._dist_to_point(p.n, p.h, p.extra["centre"])
        mask = (d >= 0.39) & (d < 0.55)
    rho = picard.solve(residual.Setup(p), p.initial_density(), 1e-12).rho
    g = np.zeros_like(rho)
    g[0][mask] = np.prod(p.h)
    return p, rho, g


def _noalloc(sol, x, g, tol=1e-12, max_iter=500):
    lib = _abi.load()
    S = sol.S
    dv = torch.empty_like(x)
    drb = (ctypes.c_double * S)()
    dsg = (ctypes.c_double * S)()
    it, res = ctypes.c_int32(), ctypes.c_double()
    st = lib.dft_adjoint_noalloc(sol.ctx, _ptr(x), _ptr(g), float(tol), int(max_iter), _ptr(dv), drb, dsg,
                                 ctypes.byref(it), ctypes.byref(res))
    _abi.check(st, "dft_adjoint_noalloc")
    return {"vext": dv, "rho_bulk": list(drb), "sigma": list(dsg), "iters": it.value, "resid": res.value}


def _rel(a, b):
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_noalloc_adjoint_equals_workspace_adjoint_twice():
    for name in ("pore32", "sphere16"):        # the second call is the smaller problem
        p, rho, g = _case(name)
        sol = from_problem(p)
        x, gd = _dev(rho), _dev(g)
        ref = sol.adjoint(x, gd, tol=1e-12)
        got = _noalloc(sol, x, gd)
        torch.cuda.synchronize()
        ev = _rel(got["vext"].cpu().numpy(), ref["vext"].cpu().numpy())
        es = _rel(got["sigma"], ref["sigma"])
        eb = _rel(got["rho_bulk"], ref["rho_bulk"])
        _say(f"  {name}: CG {got['iters']} vs {ref['iters']} iterations; rel diff vext {ev:.1e} "
             f"sigma {es:.1e} rho_b {eb:.1e}")
        assert got["iters"] == ref["iters"]
        assert ev <= 1e-12 and es <= 1e-12 and eb <= 1e-12
        sol.close()


def test_noalloc_adjoint_refuses_oversized_problems():
    p = W.charged_pore(n=64, h=0.05)
    sol = from_problem(p)
    nbytes = ctypes.c_size_t()
    _abi.check(_abi.load().dft_adjoint_workspace_size(ctypes.byref(sol.params), ctypes.byref(nbytes)), "size")
    assert nbytes.value > _abi.ADJOINT_NOALLOC_MAX_BYTES
    x = _dev(p.initial_density())
    with pytest.raises(_abi.DftError) as e:
        _noalloc(sol, x, x)
    assert e.value.status == 3   # DFT_E_WORKSPACE
