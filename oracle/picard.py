"""Picard iteration with quadratic line search, nonlinear-solver section of the paper.

The paper fixes: Picard images rho1 = G(rho0), a line-search parameter chosen by
fitting squared L2 residual norms sampled at several points with a quadratic and
taking its minimum, and the bound that keeps n3 below 0.9 (which limits the
step because n3 is linear in rho).  Everything else is a reading:

  * Step convention: rho(alpha) = rho0 + alpha (G(rho0) - rho0), i.e. alpha is the
    weight of the Picard image; the printed n3 bound is stated in that form.
  * Norm: f(alpha) = sum_i sum_fluid ((rho_i(alpha) - G_i(rho(alpha))) / rho_b_i)^2.
    Convergence when r = sqrt(f / number of fluid nodes) <= tol at the iterate.
  * A step cap c in (0, 1], starting at 1, limits alpha together with the n3
    bound: amax = min(c, bound), bound = 1 if max n3(rho(1)) <= 0.9 else
    (0.9 - max n3(rho0)) / (max n3(rho(1)) - max n3(rho0)).
    When c = 1 the full G(rho(1)) is evaluated (it is the sample at amax when
    the bound does not bind); when c < 1 only n3(rho(1)) is formed.
  * Samples f(amax/2) and f(amax); the quadratic through (0, f0), (1/2, fa),
    (1, fb) in t = alpha/amax gives t = vertex clamped to [1/100, 1] when its
    curvature is positive, else the better of t = 1/2 and t = 1 (ties to 1).
    If t is not a sample, G is evaluated there as well.
  * The best evaluated point (smallest f, ties to the larger step) is accepted
    when it lowers f, or unconditionally once amax has reached the floor
    1/1024.  After an accepted step with alpha >= c/2 the cap doubles (up to 1);
    when no point lowers f the iterate stays and c <- max(amax/4, 1/1024).
    The paper's plain fit alone lets f grow without bound for dense fluids.
  * The accepted point's G is kept for the next step.

Parity: the trajectory is a reading, pinned only by the GPU agreeing with this
code step by step; the converged density is pinned by the fixed-point
invariants in the tests (bulk fixed point, contact theorem, planar homogeneity).
"""
import numpy as np

ETA_CAP = 0.9
CAP_FLOOR = 1.0 / 1024.0


class PackingError(RuntimeError):
    pass


class PicardState:
    """rho0 with its Picard image G0, f0 = f(rho0), m0 = max n3(rho0) and the step cap."""

    def __init__(self, setup, rho0):
        self.setup = setup
        self.rho = np.array(rho0, float)
        ev = setup.evaluate(self.rho)
        self.G = ev["G"]
        self.f = setup.sqnorm(self.rho - self.G)
        self.m = ev["n3max"]
        self.cap = 1.0
        self.iters = 0
        self.rejected = 0
        self.nevals = 1
        self.npartial = 0
        self.history = []

    @property
    def r(self):
        return self.setup.residual_norm(self.f)

    def _trial(self, alpha):
        return self.rho + alpha * (self.G - self.rho)

    def _sample(self, alpha):
        x = self._trial(alpha)
        ev = self.setup.evaluate(x)
        self.nevals += 1
        return ev["G"], self.setup.sqnorm(x - ev["G"]), ev["n3max"]

    def step(self):
        """One line-search step; returns the accepted alpha or 0.0 for a rejected step."""
        cap_eta = self.setup.eta_cap
        if not self.m < cap_eta:
            raise PackingError(f"max n3 = {self.m} at the current iterate is not below {cap_eta}")
        full1 = self.cap >= 1.0
        if full1:
            G1, f1, m1 = self._sample(1.0)
        else:
            m1 = float(np.max(self.setup.weighted_densities(self._trial(1.0))[3]))
            self.npartial += 1
        bound = 1.0 if m1 <= cap_eta else (cap_eta - self.m) / (m1 - self.m)
        amax = min(self.cap, bound)
        Ga, fa, ma = self._sample(0.5 * amax)
        if full1 and amax == 1.0:
            Gb, fb, mb = G1, f1, m1
        else:
            Gb, fb, mb = self._sample(amax)
        f0 = self.f
        c2 = 2.0 * (f0 - 2.0 * fa + fb)
        c1 = fb - f0 - c2
        if c2 > 0.0:
            t = min(max(-c1 / (2.0 * c2), 0.01), 1.0)
        else:
            t = 1.0 if fb <= fa else 0.5
        cands = [(fb, 1.0, Gb, mb), (fa, 0.5, Ga, ma)]
        if t != 1.0 and t != 0.5:
            Gs, fs, ms = self._sample(t * amax)
            cands.append((fs, t, Gs, ms))
        best = cands[0]
        for c in cands[1:]:
            if c[0] < best[0] or (c[0] == best[0] and c[1] > best[1]):
                best = c
        if best[0] < f0 or amax <= CAP_FLOOR:
            alpha = best[1] * amax
            self.rho = self._trial(alpha)
            self.f, self.G, self.m = best[0], best[2], best[3]
            if alpha >= 0.5 * self.cap:
                self.cap = min(1.0, 2.0 * self.cap)
            self.iters += 1
        else:
            alpha = 0.0
            self.cap = max(0.25 * amax, CAP_FLOOR)
            self.rejected += 1
        self.history.append({"alpha": alpha, "amax": amax, "t": best[1], "r": self.r, "cap": self.cap})
        return alpha


def solve(setup, rho0, tol, max_iter=10000, callback=None):
    """Iterate until r <= tol or max_iter accepted steps; returns the PicardState."""
    st = PicardState(setup, rho0)
    while st.r > tol and st.iters < max_iter and st.rejected < 4 * max_iter + 16:
        st.step()
        if callback is not None:
            callback(st)
    return st
