#!/usr/bin/env python3
"""Benchmark of the FFT/Picard classical-DFT solver on one MI355X.

Workload (default): the 256^3 charged pore -- Ca2+/Na+/Cl- (diameters 0.2/0.2/0.362 nm,
10/100/120 mM) in a hard cylindrical pore of radius 0.7 nm lined with 8 seeded sites of
-0.5 e, h = 0.025 nm, fundamental measure theory + bulk-fluid screening + FFT Poisson.
Inputs are synthetic (seeded); the paper used no public dataset.

A "step" is one line-search Picard iteration (all its residual evaluations): the whole
hot path.  The timed window holds exactly K iterations of solves toward residual 1e-8:
solves run back to back from the bath start (dft_solve, the last one capped at the
iterations left), so it includes everything such a solve pays for -- the FP64 reference
evaluations of FP32-mixed mode, the FP64 confirmation of convergence, the status reads
between graph chunks.  W untimed iterations run the same way first.  value = those
iterations/s in FP32-mixed mode (FP32 transforms and spectral products of differences
from an FP64 reference state, FP32 difference-form FMT derivatives, FP64 n3, exponent,
norms and master density); the FP64 figure is reported beside it.  Also reported: the
steady rate of graph-launched steps past the start, per-pass HIP-event timings with
the roofline of the dominant pass, a stream-copy ceiling, and the CPU oracle timed on
one evaluation of the same 256^3 pore on the host cores.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Picard iters/s at 256³ 2-ion FMT+ES, FP32-mixed vs FP64 at 1e-8 residual"
HBM_PEAK_GBS = 8000.0


def pass_bytes(prob, fp32, compact):
    """Algorithmic HBM bytes of each pass of one plain residual evaluation.

    Every logical array is counted once per pass in which it is read or written:
    real fields of N float64 values, half spectra of N_c = nz ny (nx/2+1) complex values
    in the transform precision.  compact: the ten weighted densities leave the z pass as 7
    spectra and reach the x pass as 9, and their derivatives reach the z pass as 8 (the
    context's compact_layout).  FP64 evaluations also read setup-time spectral tables of
    N_c float64 values per row: the weight spectra w2, w3 of every species in both z passes
    and, with electrostatics, the S(S+1)/2 pair kernels in the weight pass.
    """
    nx, ny, nz = prob.n
    S = prob.nspecies
    N = nx * ny * nz
    NC = nz * ny * (nx // 2 + 1)
    R = 8 * N                         # one float64 real field
    C = NC * (8 if fp32 else 16)      # one half spectrum
    ref = S * R if fp32 else 0        # FP32-mixed: reference density read in x_fwd
    nref = 10 * 4 * N if fp32 else 0  # FP32-mixed: reference weighted densities read in x_fmt
    zin, xin, zout = (7, 9, 8) if compact else (10, 10, 10)
    T = 0 if fp32 else 8 * NC         # one FP64 table row
    es = 1 if prob.electrostatics else 0
    return {
        "x_fwd": S * R + ref + S * C,
        "y_fwd": 2 * S * C,
        "z_weights": S * C + (S + zin) * C + (2 * S + es * S * (S + 1) // 2) * T,
        "y_inv": (zin + xin) * C,
        "x_fmt": (xin + 10) * C + nref,
        "y_fwd2": (10 + zout) * C,
        "z_back_es": (zout + S) * C + S * C + 2 * S * T,
        "y_inv2": 2 * S * C,
        "x_el": S * C + 3 * S * R,
        "reduce": 0,
    }


def _solve_window(sol, rho0, iters, tol):
    """Exactly `iters` Picard iterations of solves toward tol, back to back from rho0 (the last solve
    capped at the iterations left).  Returns (seconds, number of solves, accepted, rejected, residual
    evaluations, FP64 reference evaluations, solves that reached tol)."""
    import torch
    x = rho0.clone()
    done = solves = converged = 0
    acc = {"rejected": 0, "g_evals": 0, "fp64_refresh": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < iters:
        x.copy_(rho0)
        ref0 = sol.stats()["fp64_refresh"]          # cumulative; the other counters restart per solve
        it, r, status = sol.solve(x, tol, iters - done, raise_on_fail=False)
        st = sol.stats()
        st["fp64_refresh"] -= ref0
        for k in acc:
            acc[k] += st[k]
        if it <= 0:
            raise RuntimeError(f"solve made no progress (status {status})")
        done += it
        solves += 1
        converged += int(status == 0)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, solves, done, acc["rejected"], acc["g_evals"], acc["fp64_refresh"], converged


def gpu_leg(prob, precision, steps, warmup, solve_tol, profile_reps):
    import torch
    from paper_0910_1531_amd import solver as sv

    sol = sv.from_problem(prob, precision=precision)
    rho0 = torch.tensor(prob.initial_density(), dtype=torch.float64, device="cuda")
    out = {}
    # one full solve to the configuration's tolerance from the bath start (its density is reported)
    x = rho0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref0 = sol.stats()["fp64_refresh"]
    it, r, status = sol.solve(x, solve_tol, 5000, raise_on_fail=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sol.stats()
    st["fp64_refresh"] -= ref0
    out["solve"] = {"iters": it, "seconds": t1 - t0, "its": it / (t1 - t0), "r": r, "status": status,
                    "g_evals": st["g_evals"], "rejected": st["rejected"], "fp64_refresh": st["fp64_refresh"]}
    out["rho"] = x
    # the timed window: W untimed, then exactly K timed iterations of solves toward solve_tol
    if warmup > 0:
        _solve_window(sol, rho0, warmup, solve_tol)
    dt, nsolve, acc, rej, gev, ref64, conv = _solve_window(sol, rho0, steps, solve_tol)
    out["window"] = {"seconds": dt, "iterations": acc, "solves": nsolve, "solves_converged": conv,
                     "rejected": rej, "g_evals": gev, "fp64_evals": ref64}
    out["ms_per_step"] = 1e3 * dt / steps
    out["its"] = steps / dt
    # steady stepping of the captured graph past the start (kernel-level rate, not the headline)
    y = rho0.clone()
    sol.run(y, 5)
    torch.cuda.synchronize()
    st0 = sol.stats()
    t0 = time.perf_counter()
    nrun = max(steps, 10)
    acc_run, r_run = sol.run(y, nrun)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = sol.stats()
    out["steady"] = {"steps": nrun, "seconds": t1 - t0, "its": nrun / (t1 - t0), "accepted": acc_run,
                     "rejected": st1["rejected"] - st0["rejected"], "r": r_run,
                     "g_evals": st1["g_evals"] - st0["g_evals"], "n3_evals": st1["n3_evals"] - st0["n3_evals"]}
    out["profile_ms"] = sol.profile(x, reps=profile_reps)
    out["schedule"] = sol.schedule()
    out["compact"] = bool(sol.stats()["compact_layout"])
    sol.close()
    return out


def copy_ceiling(nbytes=1 << 30, reps=20):
    """Stream-copy ceiling: torch's device copy of nbytes (read + write), timed with HIP events on the
    current stream."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _kernel_sources_sha256():
    import glob
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(root, "paper_0910_1531_amd", "csrc", "*")))
    files.append(os.path.join(root, "include", "dft.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _fit_threads(L, P, per, cap):
    t = 64
    while 2 * t <= cap and 2 * t * per <= L * P:
        t *= 2
    return t


def pass_kernel(pass_name, fp32, n, schedule, S):
    """Name of the kernel that runs the pass at n^3 (compiled length n) under the autotuned schedule,
    as rocprofv3 reports it; None for passes with several kernels or shapes not covered."""
    T = "float" if fp32 else "double"
    if pass_name == "x_fwd":
        return f"dft::k_x1c<{T}, {n}>"
    if pass_name == "x_el":
        return f"dft::k_x3c<{T}, {n}>"
    if pass_name == "x_fmt":
        if n in (16, 64, 256):   # paired-wave tiles
            return f"dft::k_x2p<{T}, {n}>"
        return f"dft::k_x2c<{T}, {n}, {1 if fp32 else 0}>"
    widths = {0: 8, 1: 4, 2: 16} if fp32 else {0: 4, 1: 2, 2: 8}
    if pass_name == "z_weights":
        v = schedule["z_weights"][1 if fp32 else 0]
        if v >= 3:
            return None   # split shapes: a plain z pass and k_z1s
        P = widths[v]
        return f"dft::k_z1c<{T}, {n}, {P}, {_fit_threads(n, P, 4, 512)}, {S}>"
    if pass_name == "z_back_es":
        P = widths[schedule["z_back"][1 if fp32 else 0]]
        return f"dft::k_z2c<{T}, {n}, {P}, {_fit_threads(n, P, 4, 512)}>"
    return None


def measured_traffic(pass_name, fp32, n, schedule, S):
    """HBM bytes per launch of the pass's kernel from the committed rocprofv3 counters
    (profiles/traffic_pore256.txt), or None when they were taken on other kernel sources."""
    want = pass_kernel(pass_name, fp32, n, schedule, S)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_pore256.txt")
    if want is None or n != 256 or not os.path.exists(path):
        return None
    sha, found = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("source_sha256 "):
                sha = line.split()[1]
            elif not line.startswith("#"):
                parts = line.rstrip("\n").split("\t")
                if len(parts) == 3 and parts[0] == want:
                    found = float(parts[1]) + float(parts[2])
    if found is None or sha != _kernel_sources_sha256():
        return None
    return found


def batch_leg():
    """The 64-point batched electrolyte workload (64^3 / 96^3 / 128^3, FP32-mixed) to 1e-8."""
    import numpy as np
    import torch
    import workloads as W
    from paper_0910_1531_amd import _abi
    from paper_0910_1531_amd.solver import Batch

    pts = W.batch_points(count=64, seed=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = Batch(pts, precision=_abi.DFT_FP32_MIXED)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    rhos = [torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda") for p in pts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, norms, sts = b.solve(rhos, 1e-8, 2000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gev = sum(b.stats(i)["g_evals"] for i in range(len(pts)))
    upd = sum(it * int(np.prod(p.n)) for it, p in zip(its, pts))
    b.close()
    sizes = [p.n[0] for p in pts]
    return {"points": len(pts), "grids": {str(n): sizes.count(n) for n in sorted(set(sizes))},
            "setup_s": round(t_setup, 3), "solve_s": round(dt, 3), "points_per_s": round(len(pts) / dt, 2),
            "iterations": {"min": int(min(its)), "median": int(np.median(its)), "max": int(max(its)),
                           "total": int(sum(its))},
            "g_evals": int(gev), "grid_point_updates_per_s": round(upd / dt, 1),
            "max_residual": float(max(norms)), "all_converged": all(s == 0 for s in sts)}


def adjoint_leg():
    """The 192^3 pore differentiation workload: forward solve to 1e-10, then the implicit adjoint
    of the Ca2+ pore occupancy (gradients w.r.t. every beta V_k(x), sigma_k and rho_b,k)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_0910_1531_amd import _abi
    from paper_0910_1531_amd import solver as sv

    p = W.config_pore(n=192, tol=1e-10)
    out = {}
    for name, prec in (("fp64", _abi.DFT_FP64), ("mixed", _abi.DFT_FP32_MIXED)):
        sol = sv.from_problem(p, precision=prec)
        x = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, r, st = sol.solve(x, 1e-10, 5000, raise_on_fail=False)
        torch.cuda.synchronize()
        out[f"forward_{name}"] = {"seconds": round(time.perf_counter() - t0, 3), "iters": it, "r": r,
                                  "status": st}
        if name == "fp64":
            mask = torch.from_numpy(W.pore_observable_mask(p)).to("cuda")
            g = torch.zeros_like(x)
            g[0][mask] = float(np.prod(p.h))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            adj = sol.adjoint(x, g, tol=1e-10)
            torch.cuda.synchronize()
            out["adjoint"] = {"seconds": round(time.perf_counter() - t0, 3), "cg_iters": adj["iters"],
                              "resid": adj["resid"], "dO_dsigma": [float(v) for v in adj["sigma"]],
                              "dO_drho_bulk": [float(v) for v in adj["rho_bulk"]]}
        sol.close()
    return out


def paper_workloads_leg():
    """The paper's own examples: the hard-sphere wall study over packing fractions (contact
    theorem error and time per solve, 384 x 16 x 16 cells of 0.00625 x 0.05 x 0.05 nm) and the
    1 M electrolyte at a hard wall (24 x 24 x 162 for the paper's 21 x 21 x 161)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_0910_1531_amd import _abi
    from paper_0910_1531_amd import solver as sv

    e1 = []
    for eta in (1e-5, 1e-4, 1e-3, 1e-2, 0.1, 0.2, 0.3):
        p = W.hs_wall_nm(eta)
        sol = sv.from_problem(p)
        b = sv.bulk(sol.params)
        x = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, r, st = sol.solve(x, 1e-10, 5000, raise_on_fail=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        m = int(round(p.radius[0] / p.h[0]))
        contact = float(x[0, 0, 0, m].item())
        e1.append({"eta": eta, "iters": it, "seconds": round(dt, 4), "status": st,
                   "contact_over_betaP_minus_1": contact / b["beta_p"] - 1.0})
        sol.close()
    p = W.electrolyte_wall()
    e2 = {"grid": list(p.n), "box_nm": list(p.extra["box"]), "paper_minutes_other_hardware": 1.5}
    for name, prec in (("fp64", _abi.DFT_FP64), ("mixed", _abi.DFT_FP32_MIXED)):
        sol = sv.from_problem(p, precision=prec)
        x = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, r, st = sol.solve(x, 1e-10, 5000, raise_on_fail=False)
        torch.cuda.synchronize()
        e2[name] = {"iters": it, "seconds": round(time.perf_counter() - t0, 4), "r": r, "status": st}
        sol.close()
    return {"e1_hard_sphere_wall": e1, "e2_electrolyte_wall": e2}


def newton_leg(n):
    """Time to solution of the pore by Newton-Krylov (FP64, exact Jacobian) from the bath start."""
    import torch
    import workloads as W
    from paper_0910_1531_amd import solver as sv

    p = W.config_pore(n=n)
    sol = sv.from_problem(p)
    x = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, cg, r, st = sol.newton(x, 1e-8, 50, raise_on_fail=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sol.close()
    return {"workload": f"charged pore {n}^3", "tol": 1e-8, "newton_steps": it, "cg_iterations": cg,
            "seconds": round(dt, 4), "r": r, "status": st}


def functionals_leg(n):
    """The pore solved to 1e-8 with each hard-sphere functional (eq. (Phi) as printed, Rosenfeld's
    original vector form, White Bear), FP64 and FP32-mixed: the cost of the functional swap."""
    import torch
    import workloads as W
    from paper_0910_1531_amd import _abi
    from paper_0910_1531_amd import solver as sv

    out = {}
    for name in ("rslt", "rosenfeld", "whitebear"):
        out[name] = {}
        for pname, prec in (("fp64", _abi.DFT_FP64), ("mixed", _abi.DFT_FP32_MIXED)):
            p = W.config_pore(n=n)
            p.hs_functional = name
            sol = sv.from_problem(p, precision=prec)
            x = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, r, st = sol.solve(x, 1e-8, 500, raise_on_fail=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out[name][pname] = {"iters": it, "seconds": round(dt, 4), "its": round(it / dt, 2), "r": r,
                                "status": st}
            sol.close()
    return out


def two_ion_leg(n, steps, warmup, tol):
    """The two-ion chemistry of the 128^3 sphere workload (1:1 RPM electrolyte, 0.3 nm ions at
    0.1 M around a charged sphere, h = 0.025 nm) at n^3: the headline's measurements for S = 2 --
    a solve from the bath to tol and the timed window of iterations -- in FP32-mixed and FP64."""
    import torch
    import workloads as W
    from paper_0910_1531_amd import _abi
    from paper_0910_1531_amd import solver as sv

    p = W.charged_sphere(n=n, h=0.025, tol=tol, name=f"sphere_{n}")
    out = {"workload": f"1:1 electrolyte (0.3 nm, 0.1 M) around a charged sphere (R 0.5 nm, -4e), {n}^3, "
                       f"h = 0.025 nm, S = 2"}
    for pname, prec in (("mixed", _abi.DFT_FP32_MIXED), ("fp64", _abi.DFT_FP64)):
        sol = sv.from_problem(p, precision=prec)
        rho0 = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
        x = rho0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, r, st = sol.solve(x, tol, 5000, raise_on_fail=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if warmup > 0:
            _solve_window(sol, rho0, warmup, tol)
        wdt, nsolve, acc, rej, gev, ref64, conv = _solve_window(sol, rho0, steps, tol)
        out[pname] = {"its": round(steps / wdt, 3), "ms_per_step": round(1e3 * wdt / steps, 4),
                      "window": {"iterations": acc, "solves": nsolve, "solves_converged": conv, "rejected": rej,
                                 "residual_evals": gev, "fp64_evals": ref64},
                      "solve_to_tol": {"iters": it, "seconds": round(dt, 4), "its": round(it / dt, 2),
                                       "r": float(f"{r:.4g}"), "status": st}}
        sol.close()
    return out


def screening_leg(n):
    """The RFD screening operator (ball averages with a radius R_SC(x) that varies over 0.3-0.6 nm)
    of the pore's three species at n^3, by Chebyshev interpolation in the radius (the paper's
    O(N^2) per-point dot product is timed on the host in cpu_baseline)."""
    import math
    import torch
    import workloads as W
    from paper_0910_1531_amd import solver as sv

    p = W.config_pore(n=n)
    f = torch.tensor(p.initial_density(), dtype=torch.float64, device="cuda")
    Rh = W.screening_radius(p, 0.3, 0.6, seed=4)
    R = torch.tensor(Rh, dtype=torch.float64, device="cuda")
    kmax = math.sqrt(sum((math.pi / hd) ** 2 for hd in p.h))
    M = min(128, int(math.ceil(kmax * (Rh.max() - Rh.min()))) + 8)
    sol = sv.from_problem(p)
    out = sol.rfd_reference(f, R, M)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        sol.rfd_reference(f, R, M, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    sol.close()
    return {"workload": f"charged pore {n}^3, 3 species, R_SC 0.3-0.6 nm", "nodes": M, "seconds": round(dt, 4)}


def screening_oracle_rate(n):
    """The oracle's O(N^2) screening operator (the paper's per-point dot product) at one grid point
    of the same n^3 workload, and that time scaled to all N points."""
    import workloads as W
    from oracle import screening

    p = W.config_pore(n=n)
    Rh = W.screening_radius(p, 0.3, 0.6, seed=4)
    t0 = time.perf_counter()
    screening.reference_at(p.initial_density(), Rh, p.n, p.h, [(0, 0, 0)])
    t = time.perf_counter() - t0
    return {"one_point_s": round(t, 2), "all_points_estimate_s": round(t * n ** 3, 0),
            "sample": f"one of the {n}^3 points (forward FFT included), scaled by N"}


def cpu_baseline(n, evals_per_iter, screening_n=None):
    """The oracle's rate on the headline workload itself: one FP64 oracle residual evaluation of the
    n^3 pore (all its threads), times the FP64 solve's residual evaluations per Picard iteration
    (the oracle's line search takes the same ones).  With screening_n, also the O(N^2) screening
    operator of the screening extra."""
    import workloads as W
    from oracle import residual

    cores = len(os.sched_getaffinity(0))
    prob = W.config_pore(n=n)
    st = residual.Setup(prob)
    rho = W.random_density(prob, seed=3, amplitude=0.3)
    t0 = time.perf_counter()
    st.evaluate(rho)
    t = time.perf_counter() - t0
    t_iter = t * evals_per_iter
    out = {"value": 1.0 / t_iter, "unit": "Picard iterations/s", "cores": cores, "kind": "oracle",
           "sample": (f"one FP64 oracle residual evaluation of the {n}^3 pore (the headline workload) took "
                      f"{t:.2f} s on {cores} threads; rate = 1 / (that time x the {evals_per_iter:.2f} "
                      f"residual evaluations per Picard iteration of the FP64 solve to 1e-8)")}
    if screening_n:
        out["rfd_screening"] = screening_oracle_rate(screening_n)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="grid nodes per axis of the pore workload")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--profile-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batch, adjoint, paper-workload, Newton, functional and screening measurements")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the per-pass HIP-event profile (for rocprofv3 runs: every launch does full work)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU; multi-GPU sharding of the grid (slab FFT with an "
              "all-to-all) is a design note only, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_0910_1531_amd import _abi

    prob = W.config_pore(n=args.n, tol=args.tol)
    if args.profile_only:
        from paper_0910_1531_amd import solver as sv
        out = {}
        for name, prec in (("mixed", _abi.DFT_FP32_MIXED), ("fp64", _abi.DFT_FP64)):
            if args.fp64_only and name == "mixed":
                continue
            sol = sv.from_problem(prob, precision=prec)
            rho = torch.tensor(prob.initial_density(), dtype=torch.float64, device="cuda")
            prof = sol.profile(rho, reps=args.profile_reps)
            pb = pass_bytes(prob, name == "mixed", bool(sol.stats()["compact_layout"]))
            out[name] = {k: {"ms": round(v, 4), "GBs": round(pb[k] / (v * 1e-3) / 1e9, 1) if v > 0 else None}
                         for k, v in prof.items()}
            sol.close()
        print(json.dumps({"profile_only": True, "workload": f"charged pore {args.n}^3", "passes": out}), flush=True)
        return
    legs = {}
    if not args.fp64_only:
        legs["mixed"] = gpu_leg(prob, _abi.DFT_FP32_MIXED, args.steps, args.warmup, args.tol, args.profile_reps)
    legs["fp64"] = gpu_leg(prob, _abi.DFT_FP64, args.steps, args.warmup, args.tol, args.profile_reps)
    head = legs["mixed"] if "mixed" in legs else legs["fp64"]
    fp32 = "mixed" in legs

    # roofline of the dominant pass of the headline precision
    prof = head["profile_ms"]
    pb = pass_bytes(prob, fp32, head["compact"])
    dom = max((k for k in prof if k != "reduce"), key=lambda k: prof[k])
    achieved = pb[dom] / (prof[dom] * 1e-3) / 1e9
    passes = {k: {"ms": round(prof[k], 4), "GB": round(pb[k] / 1e9, 4),
                  "GBs": round(pb[k] / (prof[k] * 1e-3) / 1e9, 1) if prof[k] > 0 else None} for k in prof}
    eval_ms = sum(prof.values())
    eval_gbs = sum(pb.values()) / (eval_ms * 1e-3) / 1e9
    ceiling = copy_ceiling()
    prof64 = legs["fp64"]["profile_ms"]
    pb64 = pass_bytes(prob, False, legs["fp64"]["compact"])
    eval64_ms = sum(prof64.values())
    eval64_gbs = sum(pb64.values()) / (eval64_ms * 1e-3) / 1e9

    rho_err = None
    if "mixed" in legs:
        a, b = legs["mixed"]["rho"], legs["fp64"]["rho"]
        rho_err = float(((a - b).abs().amax() / b.abs().amax()).item())

    f64 = legs["fp64"]
    s64 = f64["solve"]
    evals_per_iter = s64["g_evals"] / max(s64["iters"], 1)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.n, evals_per_iter, None if args.no_extras else args.n)
    extras = None
    if not args.no_extras:
        extras = {"two_ion_256": two_ion_leg(args.n, args.steps, args.warmup, args.tol),
                  "batch_64_points_fp32_mixed": batch_leg(), "pore192_adjoint": adjoint_leg(),
                  "paper_workloads": paper_workloads_leg(), "newton_krylov_fp64": newton_leg(args.n),
                  "hs_functionals": functionals_leg(args.n), "rfd_screening": screening_leg(args.n)}

    def window(leg):
        w = leg["window"]
        return {"iterations": w["iterations"], "solves": w["solves"], "solves_converged": w["solves_converged"],
                "rejected": w["rejected"], "residual_evals": w["g_evals"], "fp64_evals": w["fp64_evals"],
                "evals_per_step": round(w["g_evals"] / max(w["iterations"], 1), 3)}

    def steady(leg):
        s_ = leg["steady"]
        return {"its": round(s_["its"], 3), "ms_per_step": round(1e3 * s_["seconds"] / s_["steps"], 4),
                "steps": s_["steps"], "accepted": s_["accepted"], "rejected": s_["rejected"],
                "evals_per_step": round(s_["g_evals"] / s_["steps"], 3), "r_end": float(f"{s_['r']:.4g}")}

    line = {
        "metric": METRIC,
        "value": round(head["its"], 3),
        "unit": "Picard iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32-mixed: f32 transforms and spectral products of differences from an f64 reference "
                  "state, f32 difference-form FMT derivatives (log1p of the n3 change, reciprocal powers of "
                  "1 - n3); f64 n3, exponent, norms, line search and densities") if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"charged pore {args.n}^3, Ca2+/Na+/Cl- 10/100/120 mM, FMT + bulk-fluid "
                               f"electrostatics + FFT Poisson, h = 0.025 nm, solves from the bath to "
                               f"residual {args.tol:g}", "species": prob.nspecies,
                   "grid": list(prob.n), "grid_point_updates_per_s": round(head["its"] * args.n ** 3, 1)},
        "window": window(head),
        "fp64": {"value": round(f64["its"], 3), "ms_per_step": round(f64["ms_per_step"], 4), "window": window(f64)},
        "steady_state": {k: steady(v) for k, v in legs.items()},
        "solve_to_tol": {k: {kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv)
                             for kk, vv in v["solve"].items()} for k, v in legs.items()},
        "rho_rel_diff_mixed_vs_fp64": rho_err,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, fp32, args.n, head["schedule"], prob.nspecies),
                     "traffic_unit": "bytes per launch",
                     "kernel_name": pass_kernel(dom, fp32, args.n, head["schedule"], prob.nspecies),
                     "algorithmic_bytes": pb[dom], "copy_ceiling_GBs": round(ceiling, 1),
                     "frac_of_copy_ceiling": round(achieved / ceiling, 4)},
        "passes": passes,
        "eval_ms": round(eval_ms, 4),
        "eval_GBs": round(eval_gbs, 1),
        "eval_frac_of_peak": round(eval_gbs / HBM_PEAK_GBS, 4),
        "fp64_passes": {k: {"ms": round(prof64[k], 4), "GB": round(pb64[k] / 1e9, 4),
                            "GBs": round(pb64[k] / (prof64[k] * 1e-3) / 1e9, 1) if prof64[k] > 0 else None}
                        for k in prof64},
        "fp64_eval_ms": round(eval64_ms, 4),
        "fp64_eval_GBs": round(eval64_gbs, 1),
        "copy_ceiling": {"GBs": round(ceiling, 1), "what": "torch device copy of 1 GiB float64 (read + write), "
                                                           "HIP events"},
        "cpu_baseline": cpu,
        "extras": extras,
        "fft_schedule": {"shapes": {k: {"fp64": v[0], "fp32": v[1]} for k, v in head["schedule"].items()},
                         "legend": "autotuned tile shape per pass (y: inverse y of the weighted densities; y_fwd2: forward "
                                   "y of their derivatives; y_species: y passes of the species; z_plain: plain z pass); "
                                   "y passes and z_plain: 0/1/2/3/4 = 16/8/32/16/8 (FP32) or 8/4/16/8/4 (FP64) "
                                   "columns per tile, shapes 3-4 with half the threads, 5-9 the same with one LDS buffer "
                                   "instead of two; z: 0/1/2 = 8/4/16 (FP32) or 4/2/8 (FP64) columns per tile, "
                                   "z_weights 3/4/5 = the same widths after a separate plain z pass of the species"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
