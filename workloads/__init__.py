"""Seeded synthetic inputs for the FFT/Picard classical-DFT solver.

This module builds problem descriptions only: grids, species parameters, unit
conversions, external potentials (geometry) and fixed-charge densities.  It holds
none of the method's arithmetic (no weighted densities, no spectra, no bulk
thermodynamics), so both the CPU oracle and the GPU path can take their inputs
from here without sharing any computation.

Conventions shared by every consumer:
  * fields are float64 arrays laid out [species][z][y][x] (x fastest);
  * node m_d sits at x_d = m_d * h_d and the box is periodic with L_d = N_d * h_d;
  * beta_vext is beta times the external potential, +inf where a centre is excluded;
  * fixed_charge is a charge density in units of e per length-unit cubed;
  * lengths are in nm for the electrolytes and in sigma for the hard-sphere wall.

The geometries stand in for the paper's workloads (hard wall, electrolyte near a
charged object); the paper used no public dataset.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2018 exact / recommended values.
E_CHARGE = 1.602176634e-19      # C
K_BOLTZMANN = 1.380649e-23      # J/K
N_AVOGADRO = 6.02214076e23      # 1/mol
EPS0 = 8.8541878128e-12         # F/m

#: one mole per litre expressed as a number density in nm^-3
MOLAR_NM3 = N_AVOGADRO * 1e-24   # 0.602214076


def bjerrum_length_nm(temperature: float = 298.15, eps_r: float = 78.4) -> float:
    """l_B = e^2 / (4 pi eps0 eps_r k T), in nm."""
    return E_CHARGE ** 2 / (4.0 * math.pi * EPS0 * eps_r * K_BOLTZMANN * temperature) * 1e9


def molar(c: float) -> float:
    """Concentration in mol/L -> number density in nm^-3."""
    return c * MOLAR_NM3


@dataclasses.dataclass
class Problem:
    """One state point: grid, species, geometry.  All arrays float64."""
    name: str
    n: tuple            # (nx, ny, nz)
    h: tuple            # (hx, hy, hz)
    radius: np.ndarray  # [S]  R_k = sigma_k / 2
    valence: np.ndarray  # [S]
    rho_bulk: np.ndarray  # [S]
    bjerrum: float = 0.0
    electrostatics: bool = False
    beta_vext: np.ndarray | None = None     # [S, nz, ny, nx], +inf = excluded
    fixed_charge: np.ndarray | None = None  # [nz, ny, nx], e / unit^3
    tol: float = 1e-8
    eta_cap: float = 0.9
    hs_functional: str = "rslt"   # "rslt" (eq. Phi), "rosenfeld" (original vector form), "whitebear"
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def nspecies(self) -> int:
        return int(len(self.radius))

    @property
    def shape(self) -> tuple:
        nx, ny, nz = self.n
        return (nz, ny, nx)

    def initial_density(self) -> np.ndarray:
        """rho0 = rho_bulk on fluid nodes, 0 where the centre is excluded."""
        S = self.nspecies
        rho = np.empty((S,) + self.shape)
        for i in range(S):
            rho[i] = self.rho_bulk[i]
            if self.beta_vext is not None:
                rho[i][~np.isfinite(self.beta_vext[i])] = 0.0
        return rho


def node_coords(n, h):
    """Coordinates of the nodes along each axis: x_d = m_d * h_d."""
    return [np.arange(n[d]) * h[d] for d in range(3)]


def _min_image(d, L):
    return d - L * np.round(d / L)


def _dist_to_point(n, h, centre):
    """Minimum-image distance of every node to `centre`, shape [nz, ny, nx]."""
    xs = node_coords(n, h)
    L = [n[d] * h[d] for d in range(3)]
    dx = _min_image(xs[0] - centre[0], L[0])
    dy = _min_image(xs[1] - centre[1], L[1])
    dz = _min_image(xs[2] - centre[2], L[2])
    return np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)


def _axial_dist(n, h, axis_xy):
    """Minimum-image distance to a line parallel to z through (x, y) = axis_xy, [nz, ny, nx]."""
    xs = node_coords(n, h)
    L = [n[d] * h[d] for d in range(3)]
    dx = _min_image(xs[0] - axis_xy[0], L[0])
    dy = _min_image(xs[1] - axis_xy[1], L[1])
    r = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2)
    return np.broadcast_to(r[None, :, :], (n[2], n[1], n[0])).copy()


def packing_to_density(eta: float, sigma: float) -> float:
    """Number density of a one-component hard-sphere fluid with packing fraction eta."""
    return 6.0 * eta / (math.pi * sigma ** 3)


# ----------------------------------------------------------------------------- hard wall

def hard_wall(n=(32, 32, 32), h=0.2, sigma=1.0, eta=0.2, literal=False, tol=1e-10) -> Problem:
    """Hard spheres against a planar hard wall at x = 0 (periodic box).

    A centre is excluded where its minimum-image distance to the plane x = 0 is
    strictly below sigma/2, so a node exactly at contact is fluid.  With
    ``literal=True`` only 0 <= x < sigma/2 is excluded instead (one-sided slab).
    """
    if np.isscalar(h):
        h = (float(h),) * 3
    n = tuple(int(v) for v in n)
    R = 0.5 * sigma
    Lx = n[0] * h[0]
    x = np.arange(n[0]) * h[0]
    if literal:
        excl = x < R
    else:
        excl = np.minimum(x, Lx - x) < R
    bv = np.zeros((1, n[2], n[1], n[0]))
    bv[0][:, :, excl] = np.inf
    return Problem(name=f"hs_wall_{n[0]}x{n[1]}x{n[2]}", n=n, h=tuple(h),
                   radius=np.array([R]), valence=np.array([0.0]),
                   rho_bulk=np.array([packing_to_density(eta, sigma)]),
                   beta_vext=bv, tol=tol, extra={"eta": eta, "sigma": sigma})


def hs_wall_nm(eta, n=(384, 16, 16), h=(0.00625, 0.05, 0.05), radius=0.1, tol=1e-10) -> Problem:
    """Hard spheres of radius 0.1 nm against a planar hard wall at x = 0, on cells of
    0.00625 nm along the normal and 0.05 nm across it (the hard-sphere accuracy study of
    the results section), in nm.  The contact node x = R sits on the grid when R / h_x is
    an integer."""
    return hard_wall(n=n, h=h, sigma=2.0 * radius, eta=eta, tol=tol)


def electrolyte_wall(n=(24, 24, 162), box=(2.0, 2.0, 6.0), radius=(0.1, 0.2125), valence=(1.0, -1.0),
                     conc=(1.0, 1.0), lB=None, tol=1e-10, name=None) -> Problem:
    """1:1 electrolyte (cation radius 0.1 nm, anion 0.2125 nm, 1 M each) in a periodic
    2 x 2 x 6 nm cell against an uncharged hard wall at z = 0 (the ionic-fluid example of
    the results section, on a 2^a 3^b grid close to its 21 x 21 x 161).  Ion k is excluded
    where the minimum-image distance of its centre to the plane z = 0 is below R_k."""
    n = tuple(int(v) for v in n)
    h = tuple(box[d] / n[d] for d in range(3))
    R = np.asarray(radius, dtype=float)
    S = len(R)
    z = np.arange(n[2]) * h[2]
    dz = np.minimum(z, box[2] - z)
    bv = np.zeros((S, n[2], n[1], n[0]))
    for k in range(S):
        bv[k][dz < R[k], :, :] = np.inf
    return Problem(name=name or f"electrolyte_wall_{n[0]}x{n[1]}x{n[2]}", n=n, h=h, radius=R,
                   valence=np.asarray(valence, dtype=float), rho_bulk=np.array([molar(c) for c in conc]),
                   bjerrum=bjerrum_length_nm() if lB is None else lB, electrostatics=True, beta_vext=bv,
                   tol=tol, extra={"box": box})


# ----------------------------------------------------------------------------- electrolytes

def _on_node_charge(n, h, node, q):
    """Kronecker charge density: the whole charge q on one node (q / cell volume)."""
    rho_q = np.zeros((n[2], n[1], n[0]))
    rho_q[node[2], node[1], node[0]] = q / (h[0] * h[1] * h[2])
    return rho_q


def cic_charge(n, h, positions, charges):
    """Cloud-in-cell (trilinear) assignment of point charges to the periodic grid."""
    rho_q = np.zeros((n[2], n[1], n[0]))
    vol = h[0] * h[1] * h[2]
    for pos, q in zip(positions, charges):
        u = [pos[d] / h[d] for d in range(3)]
        i0 = [int(math.floor(u[d])) for d in range(3)]
        f = [u[d] - i0[d] for d in range(3)]
        for cz in (0, 1):
            wz = f[2] if cz else 1.0 - f[2]
            for cy in (0, 1):
                wy = f[1] if cy else 1.0 - f[1]
                for cx in (0, 1):
                    wx = f[0] if cx else 1.0 - f[0]
                    rho_q[(i0[2] + cz) % n[2], (i0[1] + cy) % n[1], (i0[0] + cx) % n[0]] += \
                        q * wx * wy * wz / vol
    return rho_q


def charged_sphere(n=128, h=0.025, sigma=(0.3, 0.3), valence=(1.0, -1.0), conc=(0.1, 0.1),
                   sphere_radius=0.5, sphere_charge=-4.0, lB=None, tol=1e-8, name=None) -> Problem:
    """Electrolyte around a fixed hard charged sphere centred on node (n/2, n/2, n/2).

    Ion k is excluded where |r - c| < sphere_radius + R_k (minimum image); the
    sphere's charge sits on its centre node (Kronecker density).
    """
    if np.isscalar(n):
        n = (int(n),) * 3
    if np.isscalar(h):
        h = (float(h),) * 3
    node = tuple(n[d] // 2 for d in range(3))
    centre = tuple(node[d] * h[d] for d in range(3))
    R = 0.5 * np.asarray(sigma, dtype=float)
    S = len(R)
    dist = _dist_to_point(n, h, centre)
    bv = np.zeros((S, n[2], n[1], n[0]))
    for k in range(S):
        bv[k][dist < sphere_radius + R[k]] = np.inf
    return Problem(name=name or f"sphere_{n[0]}", n=tuple(n), h=tuple(h), radius=R,
                   valence=np.asarray(valence, dtype=float),
                   rho_bulk=np.array([molar(c) for c in conc]),
                   bjerrum=bjerrum_length_nm() if lB is None else lB, electrostatics=True,
                   beta_vext=bv, fixed_charge=_on_node_charge(n, h, node, sphere_charge),
                   tol=tol, extra={"sphere_radius": sphere_radius, "sphere_charge": sphere_charge,
                                   "centre": centre})


def pore_sites(n, h, seed=3, nsites=8, pore_radius=0.7):
    """Site positions on the pore wall: theta ~ U[0, 2 pi), z ~ U[0, Lz), from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    L = [n[d] * h[d] for d in range(3)]
    cx, cy = 0.5 * L[0], 0.5 * L[1]
    theta = rng.uniform(0.0, 2.0 * math.pi, nsites)
    zpos = rng.uniform(0.0, L[2], nsites)
    return [(cx + pore_radius * math.cos(t), cy + pore_radius * math.sin(t), zz)
            for t, zz in zip(theta, zpos)]


def charged_pore(n=256, h=0.025, seed=3, nsites=8, site_charge=-0.5, pore_radius=0.7,
                 sigma=(0.2, 0.2, 0.362), valence=(2.0, 1.0, -1.0), conc=(0.010, 0.100, 0.120),
                 lB=None, tol=1e-8, name=None) -> Problem:
    """2:1 electrolyte in a hard cylindrical pore along z lined with fixed point charges.

    The pore axis runs through the box centre.  Ion k is excluded where the axial
    distance of its centre exceeds pore_radius - R_k.  The sites sit on the pore
    wall at seeded random (theta, z) and are spread to the grid by cloud-in-cell.
    """
    if np.isscalar(n):
        n = (int(n),) * 3
    if np.isscalar(h):
        h = (float(h),) * 3
    L = [n[d] * h[d] for d in range(3)]
    R = 0.5 * np.asarray(sigma, dtype=float)
    S = len(R)
    raxial = _axial_dist(n, h, (0.5 * L[0], 0.5 * L[1]))
    bv = np.zeros((S, n[2], n[1], n[0]))
    for k in range(S):
        bv[k][raxial > pore_radius - R[k]] = np.inf
    sites = pore_sites(n, h, seed=seed, nsites=nsites, pore_radius=pore_radius)
    q = cic_charge(n, h, sites, [site_charge] * nsites)
    return Problem(name=name or f"pore_{n[0]}", n=tuple(n), h=tuple(h), radius=R,
                   valence=np.asarray(valence, dtype=float),
                   rho_bulk=np.array([molar(c) for c in conc]),
                   bjerrum=bjerrum_length_nm() if lB is None else lB, electrostatics=True,
                   beta_vext=bv, fixed_charge=q, tol=tol,
                   extra={"sites": sites, "pore_radius": pore_radius, "seed": seed})


def pore_observable_mask(prob: Problem, species=0, radius=0.7, half_length=1.0):
    """Indicator of the pore region r_perp < radius and |z - z_c| < half_length (strict)."""
    n, h = prob.n, prob.h
    L = [n[d] * h[d] for d in range(3)]
    r = _axial_dist(n, h, (0.5 * L[0], 0.5 * L[1]))
    z = np.arange(n[2]) * h[2]
    zin = np.abs(z - 0.5 * L[2]) < half_length
    return (r < radius) & zin[:, None, None]


def adjoint_voxels(prob: Problem, count=32, seed=5):
    """Seeded random fluid voxels (flat [z][y][x] indices) for gradient checks."""
    rng = np.random.default_rng(seed)
    fluid = np.all(np.isfinite(prob.beta_vext), axis=0).ravel()
    idx = np.flatnonzero(fluid)
    return np.sort(rng.choice(idx, size=count, replace=False))


def batch_points(count=64, seed=4, h=0.025, sizes=(64, 96, 128), tol=1e-8):
    """Electrolyte state points with a centred charged hard sphere, drawn from default_rng(seed).

    Per point: salt 1:1 or 2:1 (p = 1/2; 2:1 means cation z = 2 at c and anion at 2c),
    c log-uniform on [0.01, 1] M, each diameter ~ U[0.2, 0.4] nm, grid N from `sizes`,
    sphere radius ~ U[0.4, 0.8] nm, sphere charge uniform integer in {-1..-6} e.
    """
    rng = np.random.default_rng(seed)
    pts = []
    for p in range(count):
        two_one = rng.uniform() < 0.5
        c = 10.0 ** rng.uniform(-2.0, 0.0)
        sig = rng.uniform(0.2, 0.4, 2)
        N = int(sizes[rng.integers(0, len(sizes))])
        srad = rng.uniform(0.4, 0.8)
        sq = -float(rng.integers(1, 7))
        if two_one:
            val, conc = (2.0, -1.0), (c, 2.0 * c)
        else:
            val, conc = (1.0, -1.0), (c, c)
        pts.append(charged_sphere(n=N, h=h, sigma=tuple(sig), valence=val, conc=conc,
                                  sphere_radius=srad, sphere_charge=sq, tol=tol,
                                  name=f"batch{p:02d}_{N}"))
    return pts


def screening_radius(prob: Problem, lo: float, hi: float, seed=0, modes=3) -> np.ndarray:
    """A smooth positive radius field [nz][ny][nx] spanning [lo, hi]: a few random low-order
    Fourier modes of the periodic box, shifted and scaled onto the interval (a stand-in for the
    local screening length R_SC(x) of the RFD electrostatics, which varies near walls and ions)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = prob.n
    x = np.arange(nx)[None, None, :] / nx
    y = np.arange(ny)[None, :, None] / ny
    z = np.arange(nz)[:, None, None] / nz
    u = np.zeros(prob.shape)
    for _ in range(modes):
        jx, jy, jz = rng.integers(0, 3, 3)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        u = u + rng.uniform(0.5, 1.0) * np.cos(2.0 * math.pi * (jx * x + jy * y + jz * z) + ph)
    u = (u - u.min()) / max(u.max() - u.min(), 1e-300)
    return lo + (hi - lo) * u


def random_density(prob: Problem, seed=0, amplitude=0.3):
    """rho = rho_bulk * mask * (1 + amplitude * u), u ~ U[-1, 1): a rough positive test field."""
    rng = np.random.default_rng(seed)
    rho = prob.initial_density()
    rho *= 1.0 + amplitude * rng.uniform(-1.0, 1.0, rho.shape)
    return rho


# The five configurations the benchmarks and tests are built on.
def config_hs_wall():
    """Hard spheres, sigma = 1, eta = 0.2, 32^3, h = sigma/5, planar wall, residual 1e-10."""
    return hard_wall(n=(32, 32, 32), h=0.2, sigma=1.0, eta=0.2, tol=1e-10)


def config_sphere_128():
    """1:1 RPM electrolyte (0.3 nm, 0.1 M), 128^3, h = 0.025 nm, sphere R = 0.5 nm, Q = -4e."""
    return charged_sphere(n=128, h=0.025, tol=1e-8, name="sphere_128")


def config_pore(n=256, tol=1e-8):
    """Ca2+/Na+/Cl- (0.2/0.2/0.362 nm; 10/100/120 mM) in a 0.7 nm pore, 8 sites of -0.5e."""
    return charged_pore(n=n, h=0.025, seed=3, tol=tol, name=f"pore_{n}")
