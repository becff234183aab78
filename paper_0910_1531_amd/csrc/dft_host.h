// Host-side pieces of the solver: parameter validation, bath thermodynamics
// (Appendix A), FFT plans and twiddle tables, and the constant block the kernels read.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dft.h"

namespace dft {

constexpr int kMaxRadices = 12;

// Mixed-radix factorization of one axis length; radices in the order the Stockham
// stages run (each in {2, 3, 4, 8}).
struct FftPlan {
    int L = 1;
    int nr = 0;
    int r[kMaxRadices] = {0};
};

// Problem constants read by every kernel (lives in device memory; uniform loads).
struct Consts {
    int S, nx, ny, nz, Kx;
    int es;                 // electrostatics on
    int cut_lambda;         // screening kernel cut at lambda_i + lambda_j (not R_i + R_j)
    long long N;            // nx * ny * nz
    long long NC;           // nz * ny * Kx (complex values per half spectrum)
    double invN;
    double dk[3];           // 2 pi / (n_d h_d)
    double h[3];
    double four_pi_lB;
    double R[DFT_MAX_SPECIES];
    double z[DFT_MAX_SPECIES];
    double rho_b[DFT_MAX_SPECIES];
    double inv_rho_b[DFT_MAX_SPECIES];
    double i4piR2[DFT_MAX_SPECIES];   // 1 / (4 pi R^2)
    double i4piR[DFT_MAX_SPECIES];    // 1 / (4 pi R)
    // bulk-fluid screening kernel of pair (i, j): C = c1 F1(Rc) + c0 F0(Rc) + cm1 Fm1(Rc)
    double sc_c1[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    double sc_c0[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    double sc_cm1[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    double sc_R[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    double nfluid;          // fluid nodes summed over species
    double eta_cap;
    // The species and pair constants of the Z1 products rounded once to FP32 (the FP32 path reads
    // them as they are instead of converting the FP64 values at every use); bath_N = N rho_b.
    double bath_N[DFT_MAX_SPECIES];
    float f_R[DFT_MAX_SPECIES], f_i4piR2[DFT_MAX_SPECIES], f_i4piR[DFT_MAX_SPECIES], f_bath_N[DFT_MAX_SPECIES];
    float f_zz[DFT_MAX_SPECIES * DFT_MAX_SPECIES];   // z_i z_j
    // The screening factor for k Rc >= 1 regrouped by sin, cos and 1 - cos (screening_hat_p):
    // with a = 4 pi c1 Rc^4, b = 4 pi c0 Rc^3, g = 4 pi cm1 Rc^2 (formed in FP64),
    // p1 = -(a + b), p2 = 2a + b, p3 = g, p4 = -2a.
    float f_sc_p1[DFT_MAX_SPECIES * DFT_MAX_SPECIES], f_sc_p2[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    float f_sc_p3[DFT_MAX_SPECIES * DFT_MAX_SPECIES], f_sc_p4[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    float f_sc_R[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    float f_four_pi_lB;
};

// Validation shared by every entry point (no HIP calls).
dft_status validate(const dft_params *p, std::string *msg);

// Appendix A bath quantities (eqs. muHSBath, HSPressure, Gamma).
dft_status bulk_info(const dft_params *p, dft_bulk_info *out, std::string *msg);

// Factor L into Stockham radices (largest first); false if L is not 1 or 2^a 3^b.
bool make_plan(int L, FftPlan *plan);

// tw[m] = exp(-2 pi i m / L), m = 0..L-1, interleaved (re, im), long-double accurate.
void twiddles(int L, std::vector<double> *out);

// Derivatives of the bath quantities with respect to rho_bulk_k and sigma_k = 2 R_k, by
// complex-step differentiation of the Appendix A formulas (exact to rounding); dGamma
// follows from implicit differentiation of eq. (Gamma).
struct BulkDeriv {
    double dmu_drho[DFT_MAX_SPECIES][DFT_MAX_SPECIES];    // [i][k]: d beta mu_i^HS / d rho_b,k
    double dmu_dsigma[DFT_MAX_SPECIES][DFT_MAX_SPECIES];  // [i][k]: d beta mu_i^HS / d sigma_k
    double dgamma_drho[DFT_MAX_SPECIES];
    double dgamma_dsigma[DFT_MAX_SPECIES];
};
void bulk_derivatives(const dft_params *p, const dft_bulk_info &b, BulkDeriv *out);

// Fill the constant block (nfluid is filled in by setup).
void fill_consts(const dft_params *p, const dft_bulk_info &b, Consts *c);

}  // namespace dft
