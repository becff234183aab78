// Launch interface of the adjoint kernels (host side).
#pragma once

#include "dft_kernels.h"

namespace dft {

// Derivative coefficients of the bulk-fluid kernel of each ordered pair (i, j) with
// respect to lambda_i and lambda_j: dC/dlambda = dc1 F1 + dc0 F0 + dcm1 Fm1.
struct AdjConsts {
    double li_c1[DFT_MAX_SPECIES * DFT_MAX_SPECIES], li_c0[DFT_MAX_SPECIES * DFT_MAX_SPECIES],
        li_cm1[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
    double lj_c1[DFT_MAX_SPECIES * DFT_MAX_SPECIES], lj_c0[DFT_MAX_SPECIES * DFT_MAX_SPECIES],
        lj_cm1[DFT_MAX_SPECIES * DFT_MAX_SPECIES];
};

struct AdjSpecArgs {
    const void *wh;   // [S] half spectra of the adjoint weights w
    const void *rh;   // [S] half spectra of rho*
    const void *dh;   // [10] half spectra of dPhi/dn at rho*
    const void *th;   // [10] half spectra of Phi''(n*) (A w)
    const AdjConsts *ac;
    double *part;     // per-block partials, width 4 + 3 * 16
};

constexpr int kAdjNV = 4 + 3 * 4 * 4;

void adj_init(long long n, const double *G, const double *g, double *w, hipStream_t s);
int adj_r0(long long n, const double *G, const double *Hw, double *r, double *p, double *part, hipStream_t s);
int adj_q(long long n, const double *G, const double *p, const double *Hp, double *q, double *part, hipStream_t s);
int adj_step(long long n, double alpha, const double *G, const double *p, const double *q, double *w, double *r,
             double *part, hipStream_t s);
void adj_dir(long long n, double beta, const double *G, const double *r, double *p, hipStream_t s);
int adj_fieldsum(long long N, int S, const double *f, double *part, hipStream_t s);
void adj_neg(long long n, const double *w, double *out, hipStream_t s);
void adj_reduce(const double *part, int nparts, int nv, double *out, hipStream_t s);
// Newton-Krylov helpers: g = (G - rho) / G on fluid nodes; per-block minima of -rho / d over
// d < 0 (returns the number of blocks); out = x + a d.
void newton_rhs(long long n, const double *G, const double *rho, double *g, hipStream_t s);
int newton_bound(long long n, const double *rho, const double *d, double *part, hipStream_t s);
void axpy(long long n, const double *x, double a, const double *d, double *out, hipStream_t s);
int adj_spec(const Geo &g, const AdjSpecArgs &a, hipStream_t s);

}  // namespace dft
