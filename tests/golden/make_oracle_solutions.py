"""Write tests/golden/oracle_solutions.{npz,json}: sampled converged densities of the FP64 CPU
oracle (oracle.picard on oracle.residual), for GPU parity tests at sizes where an oracle solve
takes minutes.

Cases (inputs from workloads, seeded):
  sphere128  the 1:1 electrolyte (0.3 nm ions at 0.1 M) around a hard sphere of radius 0.5 nm and
             charge -4 e on a 128^3 grid, h = 0.025 nm, solved to r <= 1e-12 from the bath;
  batchNN    the first point of each grid size (64^3, 96^3, 128^3) of the 64 seeded batch points,
             solved to r <= 1e-12.
Stored per case: 4096 seeded sample positions over [species][z][y][x], the x line through the
grid centre for every species, the densities there, and (JSON) the iteration count and residual.

  pore192    the charged pore (Ca2+/Na+/Cl-, 0.7 nm, 8 sites) at 192^3 solved to r <= 1e-13, then the
             oracle's implicit-adjoint gradient (oracle.adjoint) of the pore Ca2+ occupancy
             O = h^3 sum rho_Ca over r_perp < 0.7 nm, |z - z_c| < 1 nm: dO/d(beta V_k) at the 32 seeded
             voxels of every species, dO/d sigma_k and dO/d rho_bulk_k (oracle_gradient_pore192.json).

Only the oracle computes anything here.  Run: python tests/golden/make_oracle_solutions.py
(about half an hour on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import picard, residual  # noqa: E402

NSAMPLES = 4096


def sample_positions(prob, seed=11):
    """Flat indices into [S][nz][ny][nx]: NSAMPLES seeded draws, then the centre x line of each
    species (the returned order is the stored order)."""
    S = prob.nspecies
    nx, ny, nz = prob.n
    rng = np.random.default_rng(seed)
    rand = rng.choice(S * nx * ny * nz, size=NSAMPLES, replace=False)
    line = [((s * nz + nz // 2) * ny + ny // 2) * nx + np.arange(nx) for s in range(S)]
    return np.concatenate([np.sort(rand)] + line).astype(np.int64)


def cases():
    out = {"sphere128": W.config_sphere_128()}
    seen = set()
    for p in W.batch_points(count=64, seed=4):
        if p.n[0] not in seen:
            seen.add(p.n[0])
            out[f"batch{p.n[0]}"] = p
    return out


def main(only=None):
    arrays, meta = {}, {}
    npz = os.path.join(HERE, "oracle_solutions.npz")
    js = os.path.join(HERE, "oracle_solutions.json")
    if os.path.exists(npz) and only:
        with np.load(npz, allow_pickle=False) as f:
            arrays = {k: f[k] for k in f.files}
        meta = json.load(open(js))
    for name, p in cases().items():
        if only and name not in only:
            continue
        t0 = time.time()
        st = residual.Setup(p)
        ps = picard.solve(st, p.initial_density(), 1e-12, max_iter=500)
        idx = sample_positions(p)
        arrays[f"{name}_idx"] = idx
        arrays[f"{name}_rho"] = ps.rho.ravel()[idx]
        meta[name] = {"problem": p.name, "grid": list(p.n), "h": list(p.h), "iterations": ps.iters,
                      "rejected": ps.rejected, "residual": ps.r, "evaluations": ps.nevals,
                      "seconds": round(time.time() - t0, 1), "samples": int(idx.size)}
        print(name, meta[name], flush=True)
        np.savez_compressed(npz, **arrays)
        meta["_source"] = ("converged densities of the FP64 CPU oracle (Picard with the quadratic line "
                           "search), written by tests/golden/make_oracle_solutions.py")
        with open(js, "w") as fh:
            json.dump(meta, fh, indent=1, sort_keys=True)


def pore192():
    from oracle import adjoint
    t0 = time.time()
    p = W.config_pore(n=192, tol=1e-10)
    st = residual.Setup(p)
    ps = picard.solve(st, p.initial_density(), 1e-13, max_iter=500)
    print("pore192 forward", ps.iters, ps.r, round(time.time() - t0, 1), flush=True)
    mask = W.pore_observable_mask(p)
    g = np.zeros_like(ps.rho)
    g[0][mask] = float(np.prod(p.h))
    grad = adjoint.gradient(p, ps.rho, g)
    vox = W.adjoint_voxels(p, count=32, seed=5)
    out = {"_source": ("FP64 CPU oracle: Picard solve to 1e-13 and the implicit-adjoint gradient of "
                       "oracle.adjoint, written by tests/golden/make_oracle_solutions.py"),
           "problem": p.name, "grid": list(p.n), "iterations": ps.iters, "residual": ps.r,
           "observable": "h^3 sum rho_Ca over r_perp < 0.7 nm, |z - z_c| < 1 nm",
           "observable_value": float(np.sum(ps.rho[0][mask]) * np.prod(p.h)),
           "voxels": [int(v) for v in vox],
           "dO_dbetaV": [[float(grad["vext"][k].ravel()[v]) for v in vox] for k in range(p.nspecies)],
           "dO_dsigma": [float(v) for v in grad["sigma"]], "dO_drho_bulk": [float(v) for v in grad["rho_bulk"]],
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "oracle_gradient_pore192.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("pore192 gradient", out["dO_dsigma"], out["dO_drho_bulk"], out["seconds"], flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if "pore192" in args:
        args.remove("pore192")
        pore192()
    if args or not sys.argv[1:]:
        main(args or None)
