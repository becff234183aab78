"""Thin Python wrapper over the C ABI: argument marshalling only.

Every entry point has the name of its C counterpart (dft_setup -> Solver(...),
dft_residual -> Solver.residual, ...).  Device buffers are torch float64 CUDA
tensors laid out [species][z][y][x]; the workspace is a torch uint8 tensor.
"""
import ctypes

import torch

from . import _abi


def make_params(n, h, radius, valence, rho_bulk, bjerrum=0.0, electrostatics=False, precision=_abi.DFT_FP64,
                eta_cap=0.0, flags=0, hs_functional=_abi.HS_RSLT):
    """Fill a dft_params struct (hs_functional: a dft_hs_functional value or its name)."""
    p = _abi.Params()
    S = len(radius)
    for d in range(3):
        p.n[d] = int(n[d])
        p.h[d] = float(h[d])
    p.nspecies = S
    for k in range(min(S, _abi.MAX_SPECIES)):
        p.radius[k] = float(radius[k])
        p.valence[k] = float(valence[k])
        p.rho_bulk[k] = float(rho_bulk[k])
    p.bjerrum_length = float(bjerrum)
    p.electrostatics = 1 if electrostatics else 0
    p.precision = int(precision)
    p.eta_cap = float(eta_cap)
    p.flags = int(flags)
    if isinstance(hs_functional, str):
        hs_functional = _abi.HS_FUNCTIONALS[hs_functional]
    p.hs_functional = int(hs_functional)
    return p


def bulk(params):
    """dft_bulk: Appendix A bath quantities (host only)."""
    out = _abi.BulkInfo()
    _abi.check(_abi.load().dft_bulk(ctypes.byref(params), ctypes.byref(out)), "dft_bulk")
    S = params.nspecies
    return {"mu_hs": list(out.mu_hs[:S]), "beta_p": out.beta_p, "xi": list(out.xi), "gamma": out.gamma,
            "eta_msa": out.eta_msa, "omega": out.omega, "lambda": list(out.lambda_[:S]),
            "mu_es": list(out.mu_es[:S])}


def workspace_size(params):
    """dft_workspace_size (host only)."""
    b = ctypes.c_size_t()
    _abi.check(_abi.load().dft_workspace_size(ctypes.byref(params), ctypes.byref(b)), "dft_workspace_size")
    return b.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, shape, device):
    if t is None:
        return None
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    if tuple(t.shape) != tuple(shape):
        t = t.reshape(shape)
    return t.contiguous()


class Solver:
    """One problem on one GPU (dft_setup ... dft_destroy)."""

    def __init__(self, params, beta_vext=None, fixed_charge=None, device="cuda", stream=None):
        self.lib = _abi.load()
        self.params = params
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.S = params.nspecies
        nx, ny, nz = params.n[0], params.n[1], params.n[2]
        self.shape = (self.S, nz, ny, nx)
        self.N = nx * ny * nz
        self.ws = torch.empty(workspace_size(params), dtype=torch.uint8, device=self.device)
        self._vext = _dev(beta_vext, self.shape, self.device)
        self._q = _dev(fixed_charge, (nz, ny, nx), self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _abi.check(self.lib.dft_setup(ctypes.byref(params), _ptr(self._vext), _ptr(self._q), _ptr(self.ws),
                                      self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
                   "dft_setup")
        self.ctx = ctx

    def _check_rho(self, rho):
        if rho.dtype != torch.float64 or rho.device != self.device or not rho.is_contiguous() \
                or tuple(rho.shape) != self.shape:
            raise ValueError(f"rho must be a contiguous float64 {self.device} tensor of shape {self.shape}")

    def residual(self, rho, g_out=None):
        """dft_residual: (G(rho), r)."""
        self._check_rho(rho)
        if g_out is None:
            g_out = torch.empty_like(rho)
        r = ctypes.c_double()
        _abi.check(self.lib.dft_residual(self.ctx, _ptr(rho), _ptr(g_out), ctypes.byref(r)), "dft_residual")
        return g_out, r.value

    def operators(self, rho, n=True, dphi=True, c=True, phi=True):
        """dft_operators: weighted densities, dPhi/dn, exponent E and beta e phi at rho (FP64)."""
        self._check_rho(rho)
        nz, ny, nx = self.shape[1:]
        out = {}
        t = lambda k: torch.empty((k, nz, ny, nx), dtype=torch.float64, device=self.device)
        out["n"] = t(_abi.NALPHA) if n else None
        out["dphi"] = t(_abi.NALPHA) if dphi else None
        out["c"] = t(self.S) if c else None
        out["phi"] = t(1)[0] if phi else None
        _abi.check(self.lib.dft_operators(self.ctx, _ptr(rho), _ptr(out["n"]), _ptr(out["dphi"]), _ptr(out["c"]),
                                          _ptr(out["phi"])), "dft_operators")
        return out

    def set_reference(self, rho):
        self._check_rho(rho)
        _abi.check(self.lib.dft_set_reference(self.ctx, _ptr(rho)), "dft_set_reference")

    def picard_step(self, rho):
        """dft_picard_step: in place; returns (alpha, r)."""
        self._check_rho(rho)
        a, r = ctypes.c_double(), ctypes.c_double()
        _abi.check(self.lib.dft_picard_step(self.ctx, _ptr(rho), ctypes.byref(a), ctypes.byref(r)),
                   "dft_picard_step")
        return a.value, r.value

    def solve(self, rho, tol, max_iter=10000, raise_on_fail=True):
        """dft_solve: in place; returns (iterations, r, status)."""
        self._check_rho(rho)
        it, r = ctypes.c_int32(), ctypes.c_double()
        st = self.lib.dft_solve(self.ctx, _ptr(rho), float(tol), int(max_iter), ctypes.byref(it), ctypes.byref(r))
        if raise_on_fail:
            _abi.check(st, "dft_solve")
        return it.value, r.value, st

    def run(self, rho, nsteps):
        """dft_run: exactly nsteps graph-launched steps in place; returns (accepted, r)."""
        self._check_rho(rho)
        it, r = ctypes.c_int32(), ctypes.c_double()
        _abi.check(self.lib.dft_run(self.ctx, _ptr(rho), int(nsteps), ctypes.byref(it), ctypes.byref(r)), "dft_run")
        return it.value, r.value

    def profile(self, rho, reps=5):
        """dft_profile: milliseconds per pass of one residual evaluation (HIP events)."""
        self._check_rho(rho)
        ms = (ctypes.c_double * _abi.NPASS)()
        _abi.check(self.lib.dft_profile(self.ctx, _ptr(rho), int(reps), ms), "dft_profile")
        return dict(zip(_abi.PASS_NAMES, list(ms)))

    def adjoint(self, rho_star, dO_drho, tol=1e-11, max_iter=500, vext=True):
        """dft_adjoint: gradients of an observable through the fixed point rho_star.

        Returns dict with 'vext' (device [S][nz][ny][nx] or None), 'rho_bulk', 'sigma' (lists),
        'iters' and 'resid'."""
        self._check_rho(rho_star)
        g = dO_drho.contiguous()
        self._check_rho(g)
        nbytes = ctypes.c_size_t()
        _abi.check(self.lib.dft_adjoint_workspace_size(ctypes.byref(self.params), ctypes.byref(nbytes)),
                   "dft_adjoint_workspace_size")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        dv = torch.empty_like(rho_star) if vext else None
        drb = (ctypes.c_double * self.S)()
        dsg = (ctypes.c_double * self.S)()
        it, res = ctypes.c_int32(), ctypes.c_double()
        _abi.check(self.lib.dft_adjoint(self.ctx, _ptr(rho_star), _ptr(g), _ptr(ws), ws.numel(), float(tol),
                                        int(max_iter), _ptr(dv), drb, dsg, ctypes.byref(it), ctypes.byref(res)),
                   "dft_adjoint")
        return {"vext": dv, "rho_bulk": list(drb), "sigma": list(dsg), "iters": it.value, "resid": res.value}

    def newton(self, rho, tol, max_iter=100, raise_on_fail=True):
        """dft_newton: Newton-Krylov solve in place; returns (iterations, CG iterations, r, status)."""
        self._check_rho(rho)
        nbytes = ctypes.c_size_t()
        _abi.check(self.lib.dft_adjoint_workspace_size(ctypes.byref(self.params), ctypes.byref(nbytes)),
                   "dft_adjoint_workspace_size")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        it, cg, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        st = self.lib.dft_newton(self.ctx, _ptr(rho), _ptr(ws), ws.numel(), float(tol), int(max_iter),
                                 ctypes.byref(it), ctypes.byref(cg), ctypes.byref(r))
        if raise_on_fail:
            _abi.check(st, "dft_newton")
        return it.value, cg.value, r.value, st

    def rfd_reference(self, f, rsc, nodes, out=None):
        """dft_rfd_reference: ball averages of the S fields f with the radius field rsc [nz][ny][nx]."""
        self._check_rho(f)
        rsc = rsc.contiguous()
        if rsc.dtype != torch.float64 or rsc.device != self.device or tuple(rsc.shape) != tuple(f.shape[1:]):
            raise ValueError(f"rsc must be float64 {tuple(f.shape[1:])} on {self.device}")
        if out is None:
            out = torch.empty_like(f)
        _abi.check(self.lib.dft_rfd_reference(self.ctx, _ptr(f), _ptr(rsc), int(nodes), _ptr(out)),
                   "dft_rfd_reference")
        return out

    def stats(self):
        s = _abi.Stats()
        _abi.check(self.lib.dft_get_stats(self.ctx, ctypes.byref(s)), "dft_get_stats")
        return {k: getattr(s, k) for k, _ in _abi.Stats._fields_}

    def schedule(self):
        """Launch shape per tunable pass: {pass: (fp64 shape, fp32 shape)}."""
        buf = (ctypes.c_int32 * _abi.SCHEDULE_LEN)()
        _abi.check(self.lib.dft_get_schedule(self.ctx, buf), "dft_get_schedule")
        return {name: (buf[2 * i], buf[2 * i + 1]) for i, name in enumerate(_abi.TUNE_PASSES)}

    def set_schedule(self, sched):
        """Force launch shapes ({pass: (fp64 shape, fp32 shape)}, missing passes keep theirs)."""
        cur = self.schedule()
        cur.update(sched)
        buf = (ctypes.c_int32 * _abi.SCHEDULE_LEN)()
        for i, name in enumerate(_abi.TUNE_PASSES):
            buf[2 * i], buf[2 * i + 1] = cur[name]
        _abi.check(self.lib.dft_set_schedule(self.ctx, buf), "dft_set_schedule")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dft_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_problem(prob, precision=_abi.DFT_FP64, device="cuda", flags=0):
    """Build a Solver from a workloads.Problem-like object (attributes n, h, radius, ...)."""
    p = make_params(prob.n, prob.h, prob.radius, prob.valence, prob.rho_bulk, prob.bjerrum, prob.electrostatics,
                    precision, 0.0 if prob.eta_cap == 0.9 else prob.eta_cap, flags,
                    getattr(prob, "hs_functional", "rslt"))
    return Solver(p, prob.beta_vext, prob.fixed_charge, device=device)


class Batch:
    """dft_setup_batch ... dft_batch_destroy: many state points solved together."""

    def __init__(self, problems, precision=_abi.DFT_FP64, device="cuda", flags=0, stream=None):
        self.lib = _abi.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        n = len(problems)
        self.count = n
        self.params = (_abi.Params * n)()
        self.shapes = []
        self._keep = []
        vext = (ctypes.c_void_p * n)()
        qfix = (ctypes.c_void_p * n)()
        for i, prob in enumerate(problems):
            p = make_params(prob.n, prob.h, prob.radius, prob.valence, prob.rho_bulk, prob.bjerrum,
                            prob.electrostatics, precision, 0.0 if prob.eta_cap == 0.9 else prob.eta_cap, flags,
                            getattr(prob, "hs_functional", "rslt"))
            self.params[i] = p
            nx, ny, nz = prob.n
            shape = (len(prob.radius), nz, ny, nx)
            self.shapes.append(shape)
            v = _dev(prob.beta_vext, shape, self.device)
            q = _dev(prob.fixed_charge, (nz, ny, nx), self.device)
            self._keep += [v, q]
            vext[i] = v.data_ptr() if v is not None else None
            qfix[i] = q.data_ptr() if q is not None else None
        nbytes = ctypes.c_size_t()
        _abi.check(self.lib.dft_batch_workspace_size(self.params, n, ctypes.byref(nbytes)), "dft_batch_workspace_size")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _abi.check(self.lib.dft_setup_batch(self.params, n, vext, qfix, _ptr(self.ws), self.ws.numel(),
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                   "dft_setup_batch")
        self.handle = h

    def solve(self, rhos, tol, max_iter=10000, raise_on_fail=False):
        """dft_solve_batch: in place; returns (iters, norms, statuses) lists."""
        n = self.count
        for rho, shape in zip(rhos, self.shapes):
            if rho.dtype != torch.float64 or rho.device != self.device or not rho.is_contiguous() \
                    or tuple(rho.shape) != shape:
                raise ValueError("each rho must be a contiguous float64 device tensor of its point's shape")
        ptrs = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
        it = (ctypes.c_int32 * n)()
        nr = (ctypes.c_double * n)()
        st = (ctypes.c_int32 * n)()
        s = self.lib.dft_solve_batch(self.handle, ptrs, float(tol), int(max_iter), it, nr, st)
        if raise_on_fail:
            _abi.check(s, "dft_solve_batch")
        return list(it), list(nr), list(st)

    def stats(self, i):
        c = ctypes.c_void_p()
        _abi.check(self.lib.dft_batch_member(self.handle, int(i), ctypes.byref(c)), "dft_batch_member")
        s = _abi.Stats()
        _abi.check(self.lib.dft_get_stats(c, ctypes.byref(s)), "dft_get_stats")
        return {k: getattr(s, k) for k, _ in _abi.Stats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
