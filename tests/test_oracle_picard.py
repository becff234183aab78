"""Pins for oracle.picard: contact theorem, fixed-point quality, the quadratic fit on a linear map."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import picard, residual


def test_contact_theorem_on_a_fine_planar_grid():
    # Verification section, eq. (sumRule): beta P = sum_i rho_i(R_i) at a hard wall; FMT satisfies it
    # as h -> 0.  Effectively 1-D problem solved on an N x 1 x 1 grid with the contact point on a node.
    m = 768                       # h = sigma / 1536
    h = 0.5 / m
    p = W.hard_wall(n=(int(round(8.0 / h)), 1, 1), h=h, sigma=1.0, eta=0.2, tol=1e-11)
    st = residual.Setup(p)
    s = picard.solve(st, p.initial_density(), 1e-11)
    assert s.r <= 1e-11
    contact = s.rho[0, 0, 0, m]
    assert abs(contact / st.betaP - 1.0) < 1e-3
    assert s.rho[0, 0, 0, m - 1] == 0.0          # inside the wall
    mid = s.rho[0, 0, 0, p.n[0] // 2]
    assert mid == pytest.approx(p.rho_bulk[0], rel=2e-3)      # the slab centre is bulk-like


def test_contact_error_is_first_order_in_h():
    errs = []
    for m in (10, 20, 40):
        h = 0.5 / m
        p = W.hard_wall(n=(int(round(8.0 / h)), 1, 1), h=h, sigma=1.0, eta=0.2)
        st = residual.Setup(p)
        s = picard.solve(st, p.initial_density(), 1e-11)
        errs.append(s.rho[0, 0, 0, m] / st.betaP - 1.0)
    assert all(e < 0 for e in errs)
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(2.0, rel=0.05)
    # Richardson extrapolation of the first-order error lands on beta P
    assert abs(2 * errs[2] - errs[1]) < 3e-4


def test_hard_wall_32_cubed_converges_and_stays_planar():
    p = W.config_hs_wall()
    st = residual.Setup(p)
    s = picard.solve(st, p.initial_density(), p.tol, max_iter=200)
    assert s.r <= p.tol and s.iters < 100
    rho = s.rho[0]
    assert np.abs(rho - rho[:1, :1, :]).max() <= 1e-13 * rho.max()


class _LinearSetup:
    """G(rho) = A rho + b: f(alpha) is an exact quadratic, so the fitted vertex is its minimizer."""

    eta_cap = 0.9

    def __init__(self, A, b):
        self.A, self.b = A, b
        self.nfluid = len(b)

    def evaluate(self, rho):
        G = self.A @ rho + self.b
        return {"G": G, "n3max": 0.1}

    def weighted_densities(self, rho):
        return np.full((10, 1), 0.1)

    def sqnorm(self, u):
        return float(np.dot(u, u))

    def residual_norm(self, f):
        return math.sqrt(f / self.nfluid)


def test_line_search_vertex_is_exact_for_a_linear_map():
    rng = np.random.default_rng(0)
    n = 12
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = Q @ np.diag(rng.uniform(-3.0, 0.5, n)) @ Q.T      # strongly overshooting Picard map
    b = rng.normal(size=n)
    st = picard.PicardState(_LinearSetup(A, b), rng.normal(size=n))
    rho0, G0, f0 = st.rho.copy(), st.G.copy(), st.f
    d = G0 - rho0
    r0 = rho0 - G0
    Md = d - A @ d                         # residual(rho0 + a d) = r0 + a (I - A) d
    a_exact = -np.dot(r0, Md) / np.dot(Md, Md)
    assert 0.01 < a_exact < 1.0
    alpha = st.step()
    assert alpha == pytest.approx(a_exact, rel=1e-12)
    assert st.f < f0
