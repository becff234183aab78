"""Pin for oracle.adjoint: the implicit-adjoint gradient against central differences of the
observable through complete re-solves of the fixed point."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, picard, residual


def _problem():
    p = W.charged_sphere(n=16, h=0.1, sigma=(0.3, 0.24), conc=(0.5, 0.5), sphere_radius=0.25,
                         sphere_charge=-1.0)
    return p


def _observable_mask(p):
    # a shell of nodes around the sphere (species 0 only)
    d = W._dist_to_point(p.n, p.h, p.extra["centre"])
    return (d >= 0.39) & (d < 0.55)


def _solve(p, rho0=None, tol=1e-13):
    st = residual.Setup(p)
    s = picard.solve(st, p.initial_density() if rho0 is None else rho0, tol, max_iter=500)
    assert s.r <= tol
    return s.rho


def _O(p, rho, mask):
    return float(np.prod(p.h) * np.sum(rho[0][mask]))


@pytest.mark.slow
def test_adjoint_gradient_matches_finite_differences():
    p = _problem()
    mask = _observable_mask(p)
    rho = _solve(p)
    g = np.zeros_like(rho)
    g[0][mask] = np.prod(p.h)
    grad = adjoint.gradient(p, rho, g)

    # scalar parameters: rho_bulk and sigma of both species
    for field in ("rho_bulk", "sigma"):
        for k in range(2):
            base = p.rho_bulk[k] if field == "rho_bulk" else 2 * p.radius[k]
            d = 1e-4 * base
            vals = []
            for sgn in (1, -1):
                q = adjoint._perturbed(p, field, k, sgn * d)
                vals.append(_O(q, _solve(q, rho), mask))
            fd = (vals[0] - vals[1]) / (2 * d)
            got = grad[field][k]
            assert got == pytest.approx(fd, rel=2e-5, abs=1e-9 * abs(fd) + 1e-14), (field, k, got, fd)

    # external potential at two fluid voxels (one inside the observed shell)
    fluid = np.flatnonzero(np.isfinite(p.beta_vext[0]).ravel() & mask.ravel())
    for flat in (fluid[0], fluid[len(fluid) // 2]):
        for k in range(2):
            vals = []
            for sgn in (1, -1):
                q = copy.deepcopy(p)
                bv = q.beta_vext[k].reshape(-1)
                bv[flat] += sgn * 1e-3       # kT; smaller steps drown in the re-solves' own error
                vals.append(_O(q, _solve(q, rho), mask))
            fd = (vals[0] - vals[1]) / 2e-3
            got = grad["vext"][k].ravel()[flat]
            assert got == pytest.approx(fd, rel=2e-5, abs=1e-8 * np.abs(grad["vext"]).max()), (k, got, fd)
