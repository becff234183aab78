"""Pins for oracle.fmt: derivatives by complex step, bulk Percus-Yevick / Carnahan-Starling / BMCSL
identities, the White Bear factor's series against its closed form, Hessian."""
import math

import numpy as np
import pytest

from oracle import bulk, fmt, spectra


def _random_n(rng, npts, xi_big=False):
    n = np.empty((10, npts))
    n[2] = rng.uniform(0.5, 2.0, npts)
    n[0] = n[2] / (4 * math.pi * 0.25) * rng.uniform(0.8, 1.2, npts)
    n[1] = n[2] / (4 * math.pi * 0.5) * rng.uniform(0.8, 1.2, npts)
    n[3] = rng.uniform(0.01, 0.6, npts)
    v2 = rng.normal(size=(3, npts))
    scale = rng.uniform(0.05, 0.95 if not xi_big else 1.5, npts) * n[2] / np.linalg.norm(v2, axis=0)
    n[7:10] = v2 * scale
    n[4:7] = n[7:10] / (4 * math.pi * 0.5) + 0.01 * rng.normal(size=(3, npts))
    return n


@pytest.mark.parametrize("functional", fmt.FUNCTIONALS)
@pytest.mark.parametrize("xi_big", [False, True])
def test_dphi_matches_complex_step(xi_big, functional):
    rng = np.random.default_rng(1)
    n = _random_n(rng, 200, xi_big)
    n[3, :20] = np.linspace(-0.12, 0.12, 20)     # both sides of the White Bear series switch
    d = fmt.dphi(n, functional)
    for a in range(10):
        e = np.zeros_like(n)
        e[a] = 1e-30
        cs = np.imag(fmt.phi(n + 1j * e, functional)) / 1e-30
        assert np.allclose(d[a], cs, rtol=1e-13, atol=1e-13 * np.abs(cs).max() + 1e-300), a


def test_clamp_zeroes_the_tensor_term():
    rng = np.random.default_rng(2)
    n = _random_n(rng, 50)
    n[7:10] *= 3.0 * n[2] / np.linalg.norm(n[7:10], axis=0)   # |nV2| = 3 n2 > n2
    D = 1 - n[3]
    ref = -n[0] * np.log(D) + (n[1] * n[2] - np.sum(n[4:7] * n[7:10], axis=0)) / D
    assert np.allclose(fmt.phi(n), ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("rho,R", [([0.38197186342], [0.5]), ([0.02, 0.05, 0.01], [0.1, 0.1, 0.181]),
                                   ([0.3, 0.1], [0.5, 0.3])])
def test_bulk_fmt_reproduces_percus_yevick(rho, R):
    # Uniform fluid: c_i = -sum_alpha dPhi/dn_alpha w_hat_alpha^i(0) must equal -beta mu_PY_i, and
    # n0 + sum_alpha n_alpha dPhi_alpha - Phi must equal beta P_PY (Appendix A closed forms).
    rho, R = np.asarray(rho), np.asarray(R)
    n = fmt.bulk_weighted(rho, R)
    d = fmt.dphi(n[:, None])[:, 0]
    mu = np.array([d[0] + d[1] * Ri + d[2] * 4 * math.pi * Ri ** 2 + d[3] * 4 * math.pi * Ri ** 3 / 3
                   for Ri in R])
    assert np.allclose(mu, bulk.hs_mu(rho, 2 * R), rtol=1e-13)
    P = n[0] + np.dot(n, d) - fmt.phi(n[:, None])[0]
    assert P == pytest.approx(bulk.hs_pressure(rho, 2 * R), rel=1e-13)


@pytest.mark.parametrize("rho,R", [([0.38197186342], [0.5]), ([0.02, 0.05, 0.01], [0.1, 0.1, 0.181]),
                                   ([0.3, 0.1], [0.5, 0.3]), ([1e-7], [0.5])])
@pytest.mark.parametrize("functional", ["rosenfeld", "whitebear"])
def test_bulk_of_the_alternative_functionals(rho, R, functional):
    # Uniform fluid: the vector densities vanish, so Rosenfeld's original form has the same bulk as
    # eq. (Phi) (Percus-Yevick), and the White Bear form has the BMCSL bulk: Phi(bulk n) = beta f_ex,
    # sum_alpha dPhi/dn_alpha w_hat_alpha^i(0) = beta mu_ex_i and n0 + n.dPhi - Phi = beta P.
    rho, R = np.asarray(rho), np.asarray(R)
    n = fmt.bulk_weighted(rho, R)
    d = fmt.dphi(n[:, None], functional)[:, 0]
    mu = np.array([d[0] + d[1] * Ri + d[2] * 4 * math.pi * Ri ** 2 + d[3] * 4 * math.pi * Ri ** 3 / 3
                   for Ri in R])
    P = n[0] + np.dot(n, d) - fmt.phi(n[:, None], functional)[0]
    if functional == "rosenfeld":
        mu_ref, P_ref = bulk.hs_mu(rho, 2 * R), bulk.hs_pressure(rho, 2 * R)
    else:
        mu_ref, P_ref = bulk.bmcsl_mu(rho, 2 * R), bulk.bmcsl_pressure(rho, 2 * R)
        assert fmt.phi(n[:, None], functional)[0] == pytest.approx(bulk.bmcsl_free_energy(rho, 2 * R),
                                                                   rel=1e-12)
    assert np.allclose(mu, mu_ref, rtol=1e-12, atol=1e-15)
    assert P == pytest.approx(P_ref, rel=1e-12)


@pytest.mark.parametrize("eta", [1e-6, 0.05, 0.2, 0.35, 0.45])
def test_white_bear_one_component_is_carnahan_starling(eta):
    # One component: beta f_ex / rho = eta (4 - 3 eta) / (1 - eta)^2,
    # beta mu_ex = eta (8 - 9 eta + 3 eta^2) / (1 - eta)^3, beta P / rho = (1 + eta + eta^2 - eta^3) / (1 - eta)^3.
    R = 0.37
    rho = eta / (4 * math.pi * R ** 3 / 3)
    n = fmt.bulk_weighted([rho], [R])
    d = fmt.dphi(n[:, None], "whitebear")[:, 0]
    f = fmt.phi(n[:, None], "whitebear")[0]
    mu = d[0] + d[1] * R + d[2] * 4 * math.pi * R ** 2 + d[3] * 4 * math.pi * R ** 3 / 3
    assert f / rho == pytest.approx(eta * (4 - 3 * eta) / (1 - eta) ** 2, rel=1e-11)
    assert mu == pytest.approx(eta * (8 - 9 * eta + 3 * eta ** 2) / (1 - eta) ** 3, rel=1e-11)
    assert (n[0] + np.dot(n, d) - f) / rho == pytest.approx((1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3,
                                                              rel=1e-12)


def test_white_bear_factor_series_and_closed_form_agree():
    # Where both are accurate (0.1 <= |n3| <= 0.15: the 30-term series' remainder is below 1e-20 there
    # and the closed form's cancellation costs f' a few hundred ulps at |n3| = 0.1), the coefficients (k+1)(k+3)/(k+2)
    # and the closed form must give the same f and f'.  f(0) = 3/2 and f'(0) = 8/3 are the low-density
    # limits (f -> 3/2 makes the third term Rosenfeld's at n3 -> 0).
    x = np.concatenate([np.linspace(0.1, 0.15, 41), -np.linspace(0.1, 0.15, 41)])
    fs, fps = fmt.wb_factor(x, series_below=1.0)
    fc, fpc = fmt.wb_factor(x, series_below=0.0)
    assert np.allclose(fs, fc, rtol=1e-14, atol=0)
    assert np.allclose(fps, fpc, rtol=1e-13, atol=0)
    f0, fp0 = fmt.wb_factor(np.array([0.0]))
    assert f0[0] == 1.5 and fp0[0] == pytest.approx(8.0 / 3.0, rel=1e-15)
    fr, _ = fmt._third_factor(np.array([0.0]), "rosenfeld")
    assert fr[0] == 1.5


@pytest.mark.parametrize("functional", ["rosenfeld", "whitebear"])
def test_alternative_clamp_is_continuous_and_saturates(functional):
    # Beyond |nV2| = n2 the clamped third term no longer depends on nV2; at the bound it is continuous.
    rng = np.random.default_rng(4)
    n = _random_n(rng, 40)
    u = n[7:10] / np.linalg.norm(n[7:10], axis=0)

    def at(scale):
        m = n.copy()
        m[7:10] = u * scale * n[2]
        return fmt.phi(m, functional), fmt.dphi(m, functional)

    p_in, _ = at(1.0 - 1e-9)
    p_on, d_on = at(1.0 + 1e-9)
    p_far, d_far = at(3.0)
    assert np.abs(p_in - p_on).max() < 1e-7 * np.abs(p_on).max()   # a jump would not shrink with the gap
    nv1 = n[4:7]
    D = 1 - n[3]
    # the vector-2 derivative keeps only its first-order part -nV1/(1 - n3); d/dn2 no longer moves with nV2
    assert np.allclose(d_far[7:10], -nv1 / D, rtol=1e-14, atol=1e-14)
    assert np.allclose(d_on[2], d_far[2], rtol=1e-12, atol=0)


def test_fundamental_measures_c1():
    n = fmt.bulk_weighted([0.381971863421], [0.5])
    assert n[0] == pytest.approx(0.381971863421, abs=1e-12)
    assert n[1] == pytest.approx(0.190985931710, abs=1e-12)
    assert n[2] == pytest.approx(1.2, abs=1e-11)
    assert n[3] == pytest.approx(0.2, abs=1e-12)


@pytest.mark.parametrize("functional", fmt.FUNCTIONALS)
def test_hessian_vec_against_central_difference(functional):
    rng = np.random.default_rng(3)
    n = _random_n(rng, 100)
    dn = rng.normal(size=n.shape) * 1e-2 * np.abs(n).max(axis=1, keepdims=True)
    hv = fmt.hessian_vec(n, dn, functional=functional)
    eps = 1e-6
    fd = (fmt.dphi(n + eps * dn, functional) - fmt.dphi(n - eps * dn, functional)) / (2 * eps)
    assert np.allclose(hv, fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())
    # symmetry of the Hessian: u . H v = v . H u
    du = rng.normal(size=n.shape) * 1e-2
    assert np.allclose(np.sum(du * fmt.hessian_vec(n, dn, functional=functional), axis=0),
                       np.sum(dn * fmt.hessian_vec(n, du, functional=functional), axis=0), rtol=1e-10, atol=1e-14)


def _py_direct_correlation_hat(k, eta, sigma):
    """Percus-Yevick direct correlation function of one hard-sphere component (Wertheim's and
    Thiele's closed form in real space), transformed by radial quadrature:
      c(r) = -l1 - 6 eta l2 (r/sigma) - (eta/2) l1 (r/sigma)^3  for r < sigma, 0 beyond,
      l1 = (1 + 2 eta)^2 / (1 - eta)^4,  l2 = -(1 + eta/2)^2 / (1 - eta)^4."""
    from scipy.integrate import quad
    l1 = (1 + 2 * eta) ** 2 / (1 - eta) ** 4
    l2 = -(1 + eta / 2) ** 2 / (1 - eta) ** 4

    def c(r):
        x = r / sigma
        return -l1 - 6 * eta * l2 * x - 0.5 * eta * l1 * x ** 3

    return 4 * math.pi * quad(lambda r: r * r * c(r) * np.sinc(k * r / math.pi), 0.0, sigma,
                              epsabs=1e-15, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("functional", ["rslt", "rosenfeld"])
def test_linear_response_is_the_percus_yevick_direct_correlation(functional):
    # The second functional derivative of the fundamental-measure free energy of a uniform one-
    # component fluid is the Percus-Yevick direct correlation function (Rosenfeld's result): for
    # both the printed eq. (Phi) and the original vector form, whose Hessians agree at n_V = 0.
    # The oracle's residual evaluation gives it as the response of c_HS to a density kick at one
    # node, Fourier component by component.  The vector terms enter with the k-dependent factor
    # |w_V2|^2 > 0, so a wrong sign of n_V1.n_V2 / (1 - n3) or of the n2 n_V2.n_V2 term fails
    # here while every bulk identity (vectors vanish in the bulk) still holds.  Checked also:
    # the compressibility route 1 - rho c(k=0) = (1 + 2 eta)^2 / (1 - eta)^4 of the closed form.
    import workloads as W
    from oracle import residual
    eta, sigma = 0.3, 1.0
    n, h = 16, 0.25
    rho_b = 6 * eta / (math.pi * sigma ** 3)
    p = W.Problem(name="py", n=(n, n, n), h=(h, h, h), radius=np.array([sigma / 2]),
                  valence=np.zeros(1), rho_bulk=np.array([rho_b]), hs_functional=functional)
    st = residual.Setup(p)
    eps = 1e-3 * rho_b

    def E(s):
        rho = np.full((1, n, n, n), rho_b)
        rho[0, 0, 0, 0] += s * eps
        return st.evaluate(rho)["E"][0]

    dE = (-E(2) + 8 * E(1) - 8 * E(-1) + E(-2)) / (12 * eps)   # d c_HS(x) / d rho(0)
    chat = np.fft.fftn(dE).real                                 # c(k) on the mesh
    mesh = spectra.KMesh(p.n, p.h)
    k = np.broadcast_to(mesh.k, chat.shape)
    nyq = np.zeros(chat.shape, bool)
    for d in range(3):
        nyq |= np.broadcast_to(mesh.nyq[d], chat.shape)   # vector spectra are zeroed there
    ks, inv = np.unique(np.round(k[~nyq], 12), return_inverse=True)
    ref_u = np.array([_py_direct_correlation_hat(kk, eta, sigma) for kk in ks])
    ref = ref_u[inv]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(chat[~nyq] - ref)) < 1e-8 * scale
    assert 1 - rho_b * chat[0, 0, 0] == pytest.approx((1 + 2 * eta) ** 2 / (1 - eta) ** 4, rel=1e-9)
    # the k-dependence is not that of the scalar terms alone: the vector terms carry a visible part
    wv = spectra.weight_spectra(sigma / 2, mesh)
    D = 1 - eta
    vec = 2 * sum(np.abs(wv["wv2"][d]) ** 2 for d in range(3)) / (4 * math.pi * (sigma / 2) * D)
    assert np.max(np.abs(np.broadcast_to(vec, chat.shape)[~nyq])) > 1e-3 * scale
