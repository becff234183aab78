// Host-side setup math of the solver.  Plain C++ (no HIP): it is also built with g++
// and sanitizers for the host-only tests.
#include "dft_host.h"

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>

namespace dft {

static bool smooth_23(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

dft_status validate(const dft_params *p, std::string *msg) {
    char buf[256];
    if (!p) { *msg = "params is NULL"; return DFT_E_INVALID_ARG; }
    if (p->nspecies < 1 || p->nspecies > DFT_MAX_SPECIES) {
        snprintf(buf, sizeof buf, "nspecies = %d outside 1..%d", p->nspecies, DFT_MAX_SPECIES);
        *msg = buf;
        return DFT_E_UNSUPPORTED_SIZE;
    }
    for (int d = 0; d < 3; ++d) {
        int n = p->n[d];
        if (n < 1 || n > DFT_MAX_N || !smooth_23(n)) {
            snprintf(buf, sizeof buf, "n[%d] = %d is not 1 or 2^a 3^b <= %d", d, n, DFT_MAX_N);
            *msg = buf;
            return DFT_E_UNSUPPORTED_SIZE;
        }
        if (!(p->h[d] > 0.0) || !std::isfinite(p->h[d])) {
            snprintf(buf, sizeof buf, "h[%d] = %g must be positive and finite", d, p->h[d]);
            *msg = buf;
            return DFT_E_INVALID_ARG;
        }
    }
    for (int k = 0; k < p->nspecies; ++k) {
        if (!(p->radius[k] > 0.0) || !std::isfinite(p->radius[k])) {
            snprintf(buf, sizeof buf, "radius[%d] = %g must be positive", k, p->radius[k]);
            *msg = buf;
            return DFT_E_INVALID_ARG;
        }
        if (!(p->rho_bulk[k] > 0.0) || !std::isfinite(p->rho_bulk[k])) {
            snprintf(buf, sizeof buf, "rho_bulk[%d] = %g must be positive", k, p->rho_bulk[k]);
            *msg = buf;
            return DFT_E_INVALID_ARG;
        }
        if (!std::isfinite(p->valence[k])) { *msg = "valence must be finite"; return DFT_E_INVALID_ARG; }
    }
    if (p->precision != DFT_FP64 && p->precision != DFT_FP32_MIXED) {
        *msg = "precision must be DFT_FP64 or DFT_FP32_MIXED";
        return DFT_E_INVALID_ARG;
    }
    if (p->electrostatics != 0 && p->electrostatics != 1) {
        *msg = "electrostatics must be 0 or 1";
        return DFT_E_INVALID_ARG;
    }
    if (p->flags & ~(DFT_FLAG_ALLOW_NON_NEUTRAL | DFT_FLAG_CUTOFF_LAMBDA | DFT_FLAG_NO_AUTOTUNE)) {
        *msg = "unknown bits in flags";
        return DFT_E_INVALID_ARG;
    }
    if (p->hs_functional != DFT_HS_RSLT && p->hs_functional != DFT_HS_ROSENFELD &&
        p->hs_functional != DFT_HS_WHITE_BEAR) {
        *msg = "hs_functional must be DFT_HS_RSLT, DFT_HS_ROSENFELD or DFT_HS_WHITE_BEAR";
        return DFT_E_INVALID_ARG;
    }
    if (!(p->eta_cap >= 0.0 && p->eta_cap < 1.0)) {
        *msg = "eta_cap must lie in [0, 1) (0 selects 0.9)";
        return DFT_E_INVALID_ARG;
    }
    // packing fraction of the bath must be below 1
    double xi3 = 0.0;
    for (int k = 0; k < p->nspecies; ++k) xi3 += M_PI / 6.0 * p->rho_bulk[k] * std::pow(2.0 * p->radius[k], 3);
    if (!(xi3 < 1.0)) { *msg = "bulk packing fraction >= 1"; return DFT_E_INVALID_ARG; }
    if (p->electrostatics) {
        if (!(p->bjerrum_length > 0.0) || !std::isfinite(p->bjerrum_length)) {
            *msg = "bjerrum_length must be positive with electrostatics on";
            return DFT_E_INVALID_ARG;
        }
        double q = 0.0, qa = 0.0;
        for (int k = 0; k < p->nspecies; ++k) {
            q += p->valence[k] * p->rho_bulk[k];
            qa += std::fabs(p->valence[k]) * p->rho_bulk[k];
        }
        if (qa == 0.0) { *msg = "electrostatics on but no species is charged"; return DFT_E_INVALID_ARG; }
        if (!(p->flags & DFT_FLAG_ALLOW_NON_NEUTRAL) && std::fabs(q) > 1e-12 * qa) {
            snprintf(buf, sizeof buf, "bulk is not electroneutral: sum z rho = %g", q);
            *msg = buf;
            return DFT_E_NOT_NEUTRAL;
        }
    }
    return DFT_OK;
}

// ---------------------------------------------------------------- Appendix A

namespace {

struct Msa {
    double F, dF, eta, omega;
};

// Residual of eq. (Gamma) written as F = 4 Gamma^2 - 4 pi l_B sum rho X^2 and its derivative.
Msa msa_eval(double g, int S, const double *rho, const double *sig, const double *z, double lB, double Delta) {
    const double c = M_PI / (2.0 * Delta);
    double Pn = 0, dPn = 0, Om = 1, dOm = 0;
    for (int j = 0; j < S; ++j) {
        const double den = 1.0 + g * sig[j];
        Pn += rho[j] * sig[j] * z[j] / den;
        dPn -= rho[j] * sig[j] * sig[j] * z[j] / (den * den);
        Om += c * rho[j] * sig[j] * sig[j] * sig[j] / den;
        dOm -= c * rho[j] * std::pow(sig[j], 4) / (den * den);
    }
    const double eta = c * Pn / Om;
    const double deta = c * (dPn * Om - Pn * dOm) / (Om * Om);
    double sum = 0, dsum = 0;
    for (int j = 0; j < S; ++j) {
        const double den = 1.0 + g * sig[j];
        const double X = (z[j] - eta * sig[j] * sig[j]) / den;
        const double dX = (-deta * sig[j] * sig[j] * den - (z[j] - eta * sig[j] * sig[j]) * sig[j]) / (den * den);
        sum += rho[j] * X * X;
        dsum += 2.0 * rho[j] * X * dX;
    }
    Msa m;
    m.F = 4.0 * g * g - 4.0 * M_PI * lB * sum;
    m.dF = 8.0 * g - 4.0 * M_PI * lB * dsum;
    m.eta = eta;
    m.omega = Om;
    return m;
}

}  // namespace

namespace {

// Hard-sphere bath of the selected functional: beta mu_i^HS for i < S and beta P^HS, from the
// moments xi_n = pi/6 sum_k rho_k sigma_k^n.  C is double or std::complex<double> (complex
// steps of the bath derivatives).
//   Percus-Yevick (eqs. muHSBath, HSPressure; the bulk of eq. (Phi) and of Rosenfeld's form).
//   BMCSL (White Bear bulk): beta f = 6/pi [(xi2^3/xi3^2 - xi0) ln D + 3 xi1 xi2/D + xi2^3/(xi3 D^2)],
//   beta P = 6/pi [xi0/D + 3 xi1 xi2/D^2 + (3 - xi3) xi2^3/D^3], mu_i = d(beta f)/d(rho_i)
//   = sum_n a_n sigma_i^n with the a_n below (D = 1 - xi3).
template <typename C>
void hs_bath(int hs, int S, const C *rho, const C *sig, C *mu, C *bP) {
    C xi[4];
    for (int n = 0; n < 4; ++n) {
        C sum = 0.0;
        for (int k = 0; k < S; ++k) {
            C pw = 1.0;
            for (int m = 0; m < n; ++m) pw *= sig[k];
            sum += rho[k] * pw;
        }
        xi[n] = M_PI / 6.0 * sum;
    }
    const C D = 1.0 - xi[3];
    const C lD = std::log(D);
    if (hs == DFT_HS_WHITE_BEAR) {
        *bP = 6.0 / M_PI * (xi[0] / D + 3.0 * xi[1] * xi[2] / (D * D) + (3.0 - xi[3]) * xi[2] * xi[2] * xi[2] / (D * D * D));
        const C x2 = xi[2] * xi[2], x3 = xi[3];
        const C a1 = 3.0 * xi[2] / D;
        const C a2 = 3.0 * xi[1] / D + 3.0 * x2 * (lD / (x3 * x3) + 1.0 / (x3 * D * D));
        const C a3 = xi[0] / D + 3.0 * xi[1] * xi[2] / (D * D) +
                     x2 * xi[2] * (-2.0 * lD / (x3 * x3 * x3) - 1.0 / (x3 * x3 * D) - 1.0 / (x3 * x3 * D * D) +
                                   2.0 / (x3 * D * D * D));
        for (int i = 0; i < S; ++i) {
            const C s = sig[i];
            mu[i] = -lD + s * (a1 + s * (a2 + s * a3));
        }
        return;
    }
    *bP = 6.0 / M_PI * (xi[0] / D + 3.0 * xi[1] * xi[2] / (D * D) + 3.0 * xi[2] * xi[2] * xi[2] / (D * D * D));
    for (int i = 0; i < S; ++i) {
        const C s = sig[i];
        mu[i] = -lD + (3.0 * xi[2] * s + 3.0 * xi[1] * s * s) / D + 9.0 * xi[2] * xi[2] * s * s / (2.0 * D * D) +
                *bP * M_PI * s * s * s / 6.0;
    }
}

}  // namespace

dft_status bulk_info(const dft_params *p, dft_bulk_info *out, std::string *msg) {
    dft_status st = validate(p, msg);
    if (st != DFT_OK) return st;
    if (!out) { *msg = "out is NULL"; return DFT_E_INVALID_ARG; }
    std::memset(out, 0, sizeof *out);
    const int S = p->nspecies;
    double sig[DFT_MAX_SPECIES];
    for (int k = 0; k < S; ++k) sig[k] = 2.0 * p->radius[k];
    for (int n = 0; n < 4; ++n) {
        double s = 0;
        for (int k = 0; k < S; ++k) s += p->rho_bulk[k] * std::pow(sig[k], n);
        out->xi[n] = M_PI / 6.0 * s;
    }
    const double D = 1.0 - out->xi[3];
    hs_bath<double>(p->hs_functional, S, p->rho_bulk, sig, out->mu_hs, &out->beta_p);
    if (!p->electrostatics) return DFT_OK;
    const double lB = p->bjerrum_length;
    double kap2 = 0;
    for (int k = 0; k < S; ++k) kap2 += 4.0 * M_PI * lB * p->rho_bulk[k] * p->valence[k] * p->valence[k];
    // Safeguarded Newton from the Debye value kappa / 2, keeping a sign-change bracket.
    double lo = 0.0, hi = std::sqrt(kap2);
    while (msa_eval(hi, S, p->rho_bulk, sig, p->valence, lB, D).F <= 0.0) hi *= 2.0;
    double g = 0.5 * std::sqrt(kap2);
    for (int it = 0; it < 200; ++it) {
        Msa m = msa_eval(g, S, p->rho_bulk, sig, p->valence, lB, D);
        if (m.F > 0) hi = g; else lo = g;
        double gn = (m.dF != 0.0) ? g - m.F / m.dF : 0.5 * (lo + hi);
        if (!(gn > lo && gn < hi)) gn = 0.5 * (lo + hi);
        const double dg = std::fabs(gn - g);
        g = gn;
        if (dg <= 1e-15 * g) break;
    }
    Msa m = msa_eval(g, S, p->rho_bulk, sig, p->valence, lB, D);
    out->gamma = g;
    out->eta_msa = m.eta;
    out->omega = m.omega;
    for (int k = 0; k < S; ++k) {
        const double s = sig[k], zk = p->valence[k], e = m.eta;
        out->lambda[k] = p->radius[k] + 0.5 / g;
        out->mu_es[k] = -lB * (g * zk * zk / (1.0 + g * s) +
                               e * s * ((2.0 * zk - e * s * s) / (1.0 + g * s) + e * s * s / 3.0));
    }
    return DFT_OK;
}

// ---------------------------------------------------------------- bath derivatives

namespace {

using cd = std::complex<double>;

// F(Gamma) of eq. (Gamma) for complex-step arguments.
cd msa_F_c(cd g, int S, const cd *rho, const cd *sig, const double *z, double lB) {
    cd xi3 = 0.0;
    for (int k = 0; k < S; ++k) xi3 += M_PI / 6.0 * rho[k] * sig[k] * sig[k] * sig[k];
    const cd c = M_PI / (2.0 * (1.0 - xi3));
    cd Pn = 0.0, Om = 1.0;
    for (int j = 0; j < S; ++j) {
        const cd den = 1.0 + g * sig[j];
        Pn += rho[j] * sig[j] * z[j] / den;
        Om += c * rho[j] * sig[j] * sig[j] * sig[j] / den;
    }
    const cd eta = c * Pn / Om;
    cd sum = 0.0;
    for (int j = 0; j < S; ++j) {
        const cd X = (z[j] - eta * sig[j] * sig[j]) / (1.0 + g * sig[j]);
        sum += rho[j] * X * X;
    }
    return 4.0 * g * g - 4.0 * M_PI * lB * sum;
}

}  // namespace

void bulk_derivatives(const dft_params *p, const dft_bulk_info &b, BulkDeriv *out) {
    std::memset(out, 0, sizeof *out);
    const int S = p->nspecies;
    const double hstep = 1e-30;
    cd rho[DFT_MAX_SPECIES], sig[DFT_MAX_SPECIES];
    auto reset = [&]() {
        for (int k = 0; k < S; ++k) {
            rho[k] = p->rho_bulk[k];
            sig[k] = 2.0 * p->radius[k];
        }
    };
    const bool es = p->electrostatics && b.gamma > 0.0;
    double FG = 0.0;
    if (es) {
        reset();
        FG = std::imag(msa_F_c(cd(b.gamma, hstep), S, rho, sig, p->valence, p->bjerrum_length)) / hstep;
    }
    for (int k = 0; k < S; ++k) {
        for (int which = 0; which < 2; ++which) {
            reset();
            if (which == 0) rho[k] += cd(0.0, hstep);
            else sig[k] += cd(0.0, hstep);
            cd mu[DFT_MAX_SPECIES], bP;
            hs_bath<cd>(p->hs_functional, S, rho, sig, mu, &bP);
            for (int i = 0; i < S; ++i) {
                const double d = std::imag(mu[i]) / hstep;
                if (which == 0) out->dmu_drho[i][k] = d;
                else out->dmu_dsigma[i][k] = d;
            }
            if (es) {
                const double Ft = std::imag(msa_F_c(cd(b.gamma, 0.0), S, rho, sig, p->valence, p->bjerrum_length)) / hstep;
                if (which == 0) out->dgamma_drho[k] = -Ft / FG;
                else out->dgamma_dsigma[k] = -Ft / FG;
            }
        }
    }
}

// ---------------------------------------------------------------- FFT plans

bool make_plan(int L, FftPlan *plan) {
    if (L < 1 || !smooth_23(L)) return false;
    plan->L = L;
    plan->nr = 0;
    int m = L;
    while (m % 8 == 0) { plan->r[plan->nr++] = 8; m /= 8; }
    while (m % 4 == 0) { plan->r[plan->nr++] = 4; m /= 4; }
    while (m % 2 == 0) { plan->r[plan->nr++] = 2; m /= 2; }
    while (m % 3 == 0) { plan->r[plan->nr++] = 3; m /= 3; }
    return plan->nr <= kMaxRadices;
}

void twiddles(int L, std::vector<double> *out) {
    out->resize(2 * (size_t)L);
    for (int m = 0; m < L; ++m) {
        // reduce m/L to the first octant for accuracy, then evaluate in long double
        long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)L;
        (*out)[2 * m] = (double)cosl(a);
        (*out)[2 * m + 1] = (double)(-sinl(a));
    }
}

void fill_consts(const dft_params *p, const dft_bulk_info &b, Consts *c) {
    std::memset(c, 0, sizeof *c);
    c->S = p->nspecies;
    c->nx = p->n[0];
    c->ny = p->n[1];
    c->nz = p->n[2];
    c->Kx = p->n[0] / 2 + 1;
    c->es = p->electrostatics ? 1 : 0;
    c->cut_lambda = (p->flags & DFT_FLAG_CUTOFF_LAMBDA) ? 1 : 0;
    c->N = (long long)p->n[0] * p->n[1] * p->n[2];
    c->NC = (long long)c->Kx * p->n[1] * p->n[2];
    c->invN = 1.0 / (double)c->N;
    for (int d = 0; d < 3; ++d) {
        c->h[d] = p->h[d];
        c->dk[d] = 2.0 * M_PI / (p->n[d] * p->h[d]);
    }
    c->four_pi_lB = p->electrostatics ? 4.0 * M_PI * p->bjerrum_length : 0.0;
    c->eta_cap = p->eta_cap > 0.0 ? p->eta_cap : 0.9;
    const int S = p->nspecies;
    for (int k = 0; k < S; ++k) {
        c->R[k] = p->radius[k];
        c->z[k] = p->valence[k];
        c->rho_b[k] = p->rho_bulk[k];
        c->inv_rho_b[k] = 1.0 / p->rho_bulk[k];
        c->i4piR2[k] = 1.0 / (4.0 * M_PI * p->radius[k] * p->radius[k]);
        c->i4piR[k] = 1.0 / (4.0 * M_PI * p->radius[k]);
    }
    if (p->electrostatics) {
        const double lB = p->bjerrum_length;
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) {
                const double li = b.lambda[i], lj = b.lambda[j], ll = li * lj;
                const double pre = 0.5 * p->valence[i] * p->valence[j] * lB;   // z_i z_j l_B / 2
                const int ij = i * DFT_MAX_SPECIES + j;
                c->sc_c1[ij] = pre / (2.0 * ll);
                c->sc_c0[ij] = -pre * (li + lj) / ll;
                c->sc_cm1[ij] = pre * ((li - lj) * (li - lj) / (2.0 * ll) + 2.0);
                c->sc_R[ij] = (p->flags & DFT_FLAG_CUTOFF_LAMBDA) ? li + lj : p->radius[i] + p->radius[j];
            }
    }
    for (int k = 0; k < S; ++k) {
        c->bath_N[k] = (double)c->N * c->rho_b[k];
        c->f_R[k] = (float)c->R[k];
        c->f_i4piR2[k] = (float)c->i4piR2[k];
        c->f_i4piR[k] = (float)c->i4piR[k];
        c->f_bath_N[k] = (float)c->bath_N[k];
    }
    for (int ij = 0; ij < DFT_MAX_SPECIES * DFT_MAX_SPECIES; ++ij) {
        const int i = ij / DFT_MAX_SPECIES, j = ij % DFT_MAX_SPECIES;
        c->f_zz[ij] = (i < S && j < S) ? (float)(c->z[i] * c->z[j]) : 0.0f;
        const double Rc = c->sc_R[ij], R2 = Rc * Rc;
        const double a = 4.0 * M_PI * c->sc_c1[ij] * R2 * R2, bb = 4.0 * M_PI * c->sc_c0[ij] * R2 * Rc;
        c->f_sc_p1[ij] = (float)(-(a + bb));
        c->f_sc_p2[ij] = (float)(2.0 * a + bb);
        c->f_sc_p3[ij] = (float)(4.0 * M_PI * c->sc_cm1[ij] * R2);
        c->f_sc_p4[ij] = (float)(-2.0 * a);
        c->f_sc_R[ij] = (float)Rc;
    }
    c->f_four_pi_lB = (float)c->four_pi_lB;
}

}  // namespace dft
