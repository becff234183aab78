"""Host-only checks of the C ABI: symbols, bath thermodynamics, validation (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import bulk as obulk
from paper_0910_1531_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "dft.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dft_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = _declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    # and the binding wraps every one of them
    assert sorted(n for n, _ in _abi.SIGNATURES) == names


def _params(prob, **kw):
    from paper_0910_1531_amd.solver import make_params
    return make_params(prob.n, prob.h, prob.radius, prob.valence, prob.rho_bulk, prob.bjerrum,
                       prob.electrostatics, **kw)


@pytest.mark.parametrize("make", [W.config_hs_wall, W.config_sphere_128, lambda: W.config_pore(n=32)])
def test_bulk_matches_oracle(make):
    from paper_0910_1531_amd.solver import bulk
    prob = make()
    b = bulk(_params(prob))
    sig = 2 * prob.radius
    assert np.allclose(b["mu_hs"], obulk.hs_mu(prob.rho_bulk, sig), rtol=1e-14, atol=1e-16)
    assert b["beta_p"] == pytest.approx(obulk.hs_pressure(prob.rho_bulk, sig), rel=1e-14)
    if prob.electrostatics:
        g = obulk.msa_gamma(prob.rho_bulk, sig, prob.valence, prob.bjerrum)
        assert b["gamma"] == pytest.approx(g, rel=2e-15)
        assert np.allclose(b["lambda"], prob.radius + 0.5 / g, rtol=1e-14)
        assert np.allclose(b["mu_es"], obulk.msa_mu_es(prob.rho_bulk, sig, prob.valence, prob.bjerrum),
                           rtol=1e-13)


@pytest.mark.parametrize("make", [W.config_hs_wall, W.config_sphere_128, lambda: W.config_pore(n=32)])
@pytest.mark.parametrize("functional", ["rosenfeld", "whitebear"])
def test_bulk_of_the_alternative_functionals_matches_oracle(make, functional):
    # Rosenfeld's original form keeps the Percus-Yevick bath; White Bear takes the BMCSL one.
    from paper_0910_1531_amd.solver import bulk
    prob = make()
    b = bulk(_params(prob, hs_functional=functional))
    mu, bP = obulk.bath(functional, prob.rho_bulk, 2 * prob.radius)
    assert np.allclose(b["mu_hs"], mu, rtol=1e-13, atol=1e-16)
    assert b["beta_p"] == pytest.approx(bP, rel=1e-14)
    if functional == "whitebear" and obulk.moments(prob.rho_bulk, 2 * prob.radius)[3] > 0.1:
        # dense enough for Carnahan-Starling and Percus-Yevick to differ visibly (O(eta^3))
        assert not np.allclose(b["mu_hs"], obulk.hs_mu(prob.rho_bulk, 2 * prob.radius), rtol=1e-3)


def _status(fn, *args):
    return fn(*args)


def test_validation_errors_without_gpu():
    lib = _abi.load()
    prob = W.config_sphere_128()
    nbytes = ctypes.c_size_t()
    ok = _params(prob)
    assert lib.dft_workspace_size(ctypes.byref(ok), ctypes.byref(nbytes)) == 0
    assert nbytes.value > 13 * 128 ** 3 * 8
    cases = []
    p = _params(prob); p.n[0] = 100; cases.append((p, 2))            # 100 = 2^2 5^2
    p = _params(prob); p.n[1] = 2048; cases.append((p, 2))           # above the maximum
    p = _params(prob); p.nspecies = 9; cases.append((p, 2))
    p = _params(prob); p.h[2] = 0.0; cases.append((p, 1))
    p = _params(prob); p.radius[1] = -0.1; cases.append((p, 1))
    p = _params(prob); p.rho_bulk[0] = 0.0; cases.append((p, 1))
    p = _params(prob); p.rho_bulk[0] *= 1.5; cases.append((p, 8))    # not electroneutral
    p = _params(prob); p.precision = 7; cases.append((p, 1))
    p = _params(prob); p.flags = 64; cases.append((p, 1))
    p = _params(prob); p.bjerrum_length = 0.0; cases.append((p, 1))
    p = _params(prob); p.eta_cap = 1.5; cases.append((p, 1))
    p = _params(prob); p.hs_functional = 3; cases.append((p, 1))
    p = _params(prob); p.hs_functional = -1; cases.append((p, 1))
    for p, want in cases:
        assert lib.dft_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)) == want
        assert lib.dft_last_error()
    p = _params(prob, flags=_abi.FLAG_ALLOW_NON_NEUTRAL)
    p.rho_bulk[0] *= 1.5
    assert lib.dft_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)) == 0
    # setup rejects a missing or short workspace before touching the device
    ctx = ctypes.c_void_p()
    assert lib.dft_setup(ctypes.byref(ok), None, None, None, 0, None, ctypes.byref(ctx)) == 3
    assert lib.dft_setup(ctypes.byref(ok), None, None, ctypes.c_void_p(256), 16, None, ctypes.byref(ctx)) == 3
    assert lib.dft_setup(ctypes.byref(ok), None, None, ctypes.c_void_p(257), nbytes.value, None,
                         ctypes.byref(ctx)) == 3
    assert lib.dft_setup(None, None, None, None, 0, None, ctypes.byref(ctx)) == 1
    assert lib.dft_residual(None, None, None, None) == 1
    assert lib.dft_solve(None, None, 1e-8, 10, None, None) == 1
    assert lib.dft_destroy(None) == 0
    assert lib.dft_rfd_reference(None, None, None, 8, None) == 1
    assert lib.dft_adjoint(None, None, None, None, 0, 1e-10, 10, None, None, None, None, None) == 1
    assert lib.dft_adjoint_noalloc(None, None, None, 1e-10, 10, None, None, None, None, None) == 1
    assert lib.dft_last_error()


def test_all_supported_axis_lengths_validate():
    lib = _abi.load()
    nbytes = ctypes.c_size_t()
    from paper_0910_1531_amd.solver import make_params
    for n in [1, 2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 27, 32, 48, 64, 96, 128, 192, 256, 384, 512, 729, 768, 1024]:
        p = make_params((n, 1, 1), (0.1, 0.1, 0.1), [0.5], [0.0], [0.1])
        assert lib.dft_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)) == 0, n
    for n in [5, 7, 10, 100, 1536]:
        p = make_params((n, 1, 1), (0.1, 0.1, 0.1), [0.5], [0.0], [0.1])
        assert lib.dft_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)) == 2, n
