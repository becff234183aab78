"""GPU RFD screening operator (dft_rfd_reference) against the O(N^2) oracle.

The device path interpolates the ball transform in the radius on Chebyshev points; the oracle
takes the paper's per-point dot product over every wavevector.  Bars: 1e-11 of the field's
maximum once the node count exceeds k_max (max R - min R) (the geometric convergence is
checked on the way); a constant radius is exact (1e-13, one convolution).  Large grids are
checked at sampled points, which the oracle evaluates one by one.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import screening
from paper_0910_1531_amd.solver import from_problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _kmax(p):
    return math.sqrt(sum((math.pi / hd) ** 2 for hd in p.h))


def _problem(n, S, h=(0.1, 0.12, 0.09)):
    R = np.array([0.16, 0.11, 0.2])[:S]
    return W.Problem(name=f"screen{n}", n=tuple(n), h=tuple(h), radius=R, valence=np.zeros(S),
                     rho_bulk=np.full(S, 0.8))


# run-time-length kernels, compiled lengths, and a mix
@pytest.mark.parametrize("n,S", [((12, 8, 9), 2), ((16, 16, 16), 1), ((24, 8, 32), 3)])
def test_matches_the_per_point_dot_product(n, S):
    p = _problem(n, S)
    f = W.random_density(p, seed=7, amplitude=0.5)
    f[:, :, :, :2] = 0.0                          # a wall-like jump
    R = W.screening_radius(p, 0.12, 0.35, seed=2)
    ref = screening.reference(f, R, p.n, p.h)
    sol = from_problem(p)
    scale = np.abs(ref).max()
    errs = {}
    M_conv = int(math.ceil(_kmax(p) * (R.max() - R.min()))) + 8
    for M in (4, 8, 16, M_conv):
        out = sol.rfd_reference(_dev(f), _dev(R), M)
        errs[M] = float(np.abs(out.cpu().numpy() - ref).max() / scale)
    _say(f"screening n={n} S={S}: k_max dR = {_kmax(p) * (R.max() - R.min()):.1f}; errors by node count: "
         + " ".join(f"{m}:{e:.1e}" for m, e in errs.items()))
    assert errs[M_conv] < 1e-11
    assert errs[8] < errs[4] and errs[16] < errs[8]


@pytest.mark.parametrize("precision", [0, 1])
def test_constant_radius_is_one_convolution(precision):
    # FP64 arithmetic in either precision of the context
    p = _problem((16, 12, 18), 2)
    f = W.random_density(p, seed=8, amplitude=0.5)
    R = np.full(p.shape, 0.23)
    want = screening.convolution(f, 0.23, p.n, p.h)
    sol = from_problem(p, precision=precision)
    for M in (1, 7):
        out = sol.rfd_reference(_dev(f), _dev(R), M).cpu().numpy()
        assert np.abs(out - want).max() < 1e-13 * np.abs(want).max()


def test_in_place_and_argument_errors():
    from paper_0910_1531_amd import _abi
    p = _problem((16, 16, 16), 2)
    f = W.random_density(p, seed=9, amplitude=0.5)
    R = W.screening_radius(p, 0.15, 0.3, seed=3)
    sol = from_problem(p)
    x = _dev(f)
    a = sol.rfd_reference(x, _dev(R), 24).cpu().numpy()
    sol.rfd_reference(x, _dev(R), 24, out=x)      # f_ref aliasing f
    assert np.array_equal(x.cpu().numpy(), a)
    lib = sol.lib
    import ctypes
    ptr = ctypes.c_void_p
    bad = R.copy()
    bad[3, 4, 5] = 0.0
    xb, rb = _dev(f), _dev(bad)
    assert lib.dft_rfd_reference(sol.ctx, ptr(xb.data_ptr()), ptr(rb.data_ptr()), 8, ptr(xb.data_ptr())) == 1
    rg = _dev(R)
    assert lib.dft_rfd_reference(sol.ctx, ptr(xb.data_ptr()), ptr(rg.data_ptr()), 0, ptr(xb.data_ptr())) == 1
    assert lib.dft_rfd_reference(sol.ctx, ptr(xb.data_ptr()), ptr(rg.data_ptr()), _abi.RFD_MAX_NODES + 1,
                                 ptr(xb.data_ptr())) == 1
    # the Picard state is kept: a residual after the call equals one before it
    g1, r1 = sol.residual(_dev(f))
    sol.rfd_reference(_dev(f), _dev(R), 8)
    g2, r2 = sol.residual(_dev(f))
    assert r1 == r2 and torch.equal(g1, g2)


def test_pore128_sampled_points():
    # The pore electrolyte's grid (h = 0.025 nm, 3 species) at 128^3 with R_SC spanning 0.3-0.6 nm.
    p = W.config_pore(n=128)
    f = p.initial_density()
    R = W.screening_radius(p, 0.3, 0.6, seed=4)
    M = int(math.ceil(_kmax(p) * (R.max() - R.min()))) + 8
    sol = from_problem(p)
    out = sol.rfd_reference(_dev(f), _dev(R), M).cpu().numpy()
    rng = np.random.default_rng(5)
    pts = [tuple(int(v) for v in rng.integers(0, 128, 3)) for _ in range(4)]
    pts.append(tuple(int(v) for v in np.unravel_index(np.argmin(R), R.shape)))
    pts.append(tuple(int(v) for v in np.unravel_index(np.argmax(R), R.shape)))
    want = screening.reference_at(f, R, p.n, p.h, pts)
    got = np.array([[out[i][q] for q in pts] for i in range(f.shape[0])])
    err = np.abs(got - want).max() / np.abs(f).max()
    _say(f"pore128: {M} nodes, max error at {len(pts)} sampled points {err:.1e}")
    assert err < 1e-11


def test_picard_run_continues_across_the_screening_call():
    # The screening operator borrows the line-search buffers that do not hold the current iterate,
    # so a Picard run continued after it equals one without it (the buffers' roles have rotated
    # during the first steps).
    p = W.charged_sphere(n=32, h=0.1)
    a, b = from_problem(p), from_problem(p)
    xa = _dev(p.initial_density())
    xb = xa.clone()
    a.run(xa, 4)
    b.run(xb, 4)
    R = W.screening_radius(p, 0.3, 0.6, seed=1)
    b.rfd_reference(_dev(p.initial_density()), _dev(R), 8)
    acc_a, ra = a.run(xa, 4)
    acc_b, rb = b.run(xb, 4)
    _say(f"sphere32: 4 + 4 steps, accepted {acc_a} / {acc_b}, r {ra:.3e} / {rb:.3e}")
    assert acc_a == acc_b and ra == rb and torch.equal(xa, xb)
