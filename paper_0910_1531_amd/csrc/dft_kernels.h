// Launch interface of the pass kernels (host side).  Every launcher checks the tile
// shape against the kernel's compile-time capacity before launching.
#pragma once

#include <hip/hip_runtime.h>

#include "dft_device.h"

namespace dft {

// Line-search and status scalars kept in device memory (graph-capturable control).
struct DevState {
    double f0, m0;          // current iterate: f = ||rho - G(rho)||_w^2, max n3
    double f1, m1;          // at alpha = 1 (full G, or n3 only)
    double fa, ma, fb, mb, fs, ms;
    double amax, t, alpha_trial, alpha_acc, cap, alpha_zero, alpha_one;
    double r, tol, nfluid, eta_cap;
    double best_f;
    long long iters, rejected, gevals, n3evals, max_iter;
    int gate_full1, gate_part1, gate_a, gate_b, gate_s, gate_run, gate_one;
    int gate_refresh;       // batches: this problem takes the next FP64 reference evaluation
    int src;                // accepted sample: 0 = amax, 1 = amax/2, 2 = vertex
    int status;             // dft_status of the device loop (NONFINITE, PACKING)
    int converged;
    int sel;                // role of the current iterate's buffers (Roles); accepted samples rotate it
};

// Pointers every pass kernel needs (device memory inside the workspace).
struct Geo {
    const Consts *cs;
    DevPlan px, py, pz;
    const void *tw64[3];   // cx<double> tables per axis
    const void *tw32[3];   // cx<float> tables per axis
    int nx, ny, nz, Kx, S;
    int es;                // electrostatics on (mirrors Consts::es for launch choices)
    int cut_lambda;        // screening cutoff at lambda_i + lambda_j (mirrors Consts::cut_lambda)
    // Compact vector layout between the z and y passes (every pass on compiled-length kernels):
    // the x and y components of a vector density differ from one field by -i k_x and -i k_y, so
    // Z1 writes n0..n3, the nV1 sum and the two z components (slots 0-4, 6, 9), the inverse y
    // pass expands them to nine fields (all but nV2_x) and X2 forms nV2_x = -i k_x n3 itself; X2
    // multiplies the x components of the derivatives by i k_x, the forward y pass folds the y
    // components in (slots 0-4, 6, 7, 9) and Z2 reads those.
    int compact = 0;
    long long N, NC;
    // Batches of identically shaped problems: the kernels of one launch cover nprob
    // problems whose workspaces sit pstride bytes apart (blockIdx.z carries the problem).
    int nprob = 1;
    long long pstride = 0;
    // FP64 spectral tables of the compiled-length z kernels, [row][z][y][kx] (null: none):
    // rows 0..S-1 w2_s(k), S..2S-1 w3_s(k), then with electrostatics the
    // screening-minus-Coulomb kernel K_ij(k) of each pair i <= j.
    const double *tab64 = nullptr;
    int ntab = 0;
    // Launch shape of the compiled-length kernels per tunable pass and precision
    // ([pass][0] FP64, [pass][1] FP32); 0 is the default shape.
    int tune[DFT_TUNE_PASSES][2] = {};
};

// Passes whose launch shape the autotuner picks.
// Tunable passes: the inverse y pass of the ten weighted-density spectra, the plain z pass, Z1,
// Z2, the forward y pass of the ten derivative spectra, the y passes of the species spectra.
enum TunePass { TUNE_Y = 0, TUNE_YZ = 1, TUNE_Z1 = 2, TUNE_Z2 = 3, TUNE_YF = 4, TUNE_YS = 5 };

// Where the reductions of one residual evaluation go.
struct RedBufs {
    double *fpart;   // per-block partial sums of the weighted residual (X3)
    double *mpart;   // per-block partial maxima of n3 (X2)
    int *fflag;      // per-block flags of X3: 1 = non-finite
    int *mflag;      // per-block flags of X2: 1 = non-finite evaluation, 2 = xi^2 clamp used,
                     // 4 = non-finite n3 (only then is the n3 maximum +inf)
    int cap;         // capacity of each array
};

enum XFwdMode { XF_PLAIN = 0, XF_TRIAL = 1 };
enum X2Mode { X2_FULL = 0, X2_N3_ONLY = 1, X2_HESS = 2 };
enum Z2Mode { Z2_EL = 0, Z2_POISSON = 1, Z2_BALL = 2 };

// Rotating buffers of the line search (one set per problem): densities rho[k] and Picard images
// G[k], k = 0..3.  The current iterate and its image sit in role *sel; the sample of kind q
// (ROLE_B: alpha = amax, or 1; ROLE_A: amax / 2; ROLE_S: the fitted step) writes its trial
// density and image to role (*sel + 1 + q) mod 4, so accepting a sample moves *sel instead of
// copying the arrays.  ROLE_PRIME evaluates the iterate itself (image into role *sel); ROLE_N3
// forms the trial point at alpha without writing it.
enum RoleKind { ROLE_B = 0, ROLE_A = 1, ROLE_S = 2, ROLE_PRIME = 3, ROLE_N3 = 4 };
struct Roles {
    double *rho[4];
    double *G[4];
    const int *sel;           // null: the plain pointers of the pass arguments are used
};

struct XFwdArgs {
    const double *src;        // [S][N] input (plain) or rho0 (trial)
    const double *g0;         // [S][N] Picard image (trial)
    const double *alpha;      // device scalar (trial)
    double *rho_t;            // [S][N] trial point out (trial), may be null
    const double *ref;        // [S][N] FP32-mixed reference density (subtracted), may be null
    void *spec;               // [S] half spectra out
    int nfield;               // fields to transform
    int mode;
    const int *gate;
    Roles roles;              // trial mode with roles.sel: src, g0 and rho_t from the roles (kind)
    int kind;
};

struct YArgs {
    void *spec;
    int nfield;
    int dir;
    const int *gate;
    int axis = 1;       // 1: y, 2: z (plain transform along z)
    int vec = 0;        // compact vector layout of specB (Geo::compact): 1 inverse (7 -> 9 fields),
                        // 2 forward (10 -> 8 fields); 0 plain
};

struct Z1Args {
    void *specA;        // [S] in (after x, y forward); out with electrostatics: the unnormalized
                        // electrostatic spectra sum_j (C_ij - z_i z_j 4 pi l_B / D) rho_hat_j
    void *specB;        // [10] out: n_alpha half spectra after inverse z (x invN)
    int n3only;         // only n3 into specB[0]
    int diff;           // FP32-mixed difference evaluation: no bath subtraction
    const int *gate;
};

struct Z2Args {
    void *specB;        // [10] dPhi/dn half spectra after x, y forward
    void *specA;        // [S] in: electrostatic spectra from Z1; out: E_hat after inverse z (x invN)
    int mode;           // Z2_EL, Z2_POISSON or Z2_BALL
    int nsrc;           // Z2_POISSON, Z2_BALL: number of source fields in specA
    double wsrc[DFT_MAX_SPECIES];   // Z2_POISSON: weights of the sources
    double radius;      // Z2_BALL: specB[i] = specA[i] x ball_mean(|k|, radius) / N (z transformed)
    const int *gate;
};

struct X2Args {
    void *specB;              // [10] in: n half spectra after y inverse; out: dPhi spectra
    int mode;
    const float *nref;        // FP32-mixed: reference weighted densities [10][N]
    float *nref_out;          // FP64 refresh: write n rounded to float [10][N]
    double *n_out;            // [10][N] FP64 copies for inspection, may be null
    double *dphi_out;         // [10][N], may be null
    const double *nstar;      // X2_HESS: weighted densities of the expansion point [10][N] (FP64)
    double *t_out;            // X2_HESS: Phi''(nstar) n written as [10][N] FP64, may be null
    int hs;                   // dft_hs_functional (the FP32 difference form covers DFT_HS_RSLT only)
    RedBufs red;
    const int *gate;
};

struct X3Args {
    void *specA;              // [S] E_hat half spectra after y inverse
    int nfield;
    int raw;                  // write E (+ addend) only
    const double *addend;     // raw mode: added to E (may be null)
    double *raw_out;          // raw mode output [nfield][N]
    const double *base;       // [S][N] exponent base (beta mu_b - beta V - z beta e phi_fixed [+ E_ref])
    const double *rho_t;      // [S][N] point of evaluation (residual)
    double *g_out;            // [S][N] G(rho_t), may be null
    double *e_out;            // [S][N] E for inspection, may be null
    const double *e_phi;      // with e_out: beta e phi_fixed, subtracted z_k times from E (may be null)
    double *lp_out;           // FP64 refresh: base + E, may be null
    RedBufs red;
    const int *gate;
    Roles roles;              // with roles.sel: rho_t and g_out from the roles (kind)
    int kind;
};

// Launchers (precision T = double or float of the transforms).
template <typename T> void launch_x_forward(const Geo &g, const XFwdArgs &a, hipStream_t s);
template <typename T> void launch_y(const Geo &g, const YArgs &a, hipStream_t s);
// Compiled-length kernels (ct_launch_*.hip); false when the length has none.
template <typename T> bool launch_y_ct(const Geo &g, const YArgs &a, hipStream_t s);
template <typename T> bool launch_z1_ct(const Geo &g, const Z1Args &a, int es, hipStream_t s);
template <typename T> bool launch_z2_ct(const Geo &g, const Z2Args &a, hipStream_t s);
template <typename T> int launch_x2_ct(const Geo &g, const X2Args &a, hipStream_t s);   // blocks, 0: none
template <typename T> bool launch_x2_alt_ct(const Geo &g, const X2Args &a, hipStream_t s);
template <typename T> bool launch_x1_ct(const Geo &g, const XFwdArgs &a, hipStream_t s);
template <typename T> bool launch_x3_ct(const Geo &g, const X3Args &a, hipStream_t s);
int x_ct_pairs(int nx);        // row pairs per block of the compiled-length x kernels, 0 if none
int x2_ct_min_pairs(int nx);   // fewest row pairs per block of the length's x2 kernels, 0 if none
int y_ct_variants(int L, bool fp32);   // launch shapes of the y kernels of length L (0: none)
int z_ct_variants(int L);              // launch shapes of the z kernels of length L (0: none)
int z1_ct_variants(int L);             // launch shapes of the Z1 pass (fused and split)
// Rows of the spectral tables for S species (0 when the compiled z kernels cannot run).
int spec_table_rows(int nz, int S, int es);
// Fill g.tab64 from the constants and twiddle tables.
void launch_spec_tables(const Geo &g, hipStream_t s);
template <typename T> void launch_z1(const Geo &g, const Z1Args &a, hipStream_t s);
template <typename T> void launch_z2(const Geo &g, const Z2Args &a, hipStream_t s);
template <typename T> int launch_x2(const Geo &g, const X2Args &a, hipStream_t s);   // returns the blocks
template <typename T> void launch_x3(const Geo &g, const X3Args &a, hipStream_t s);

// Number of blocks the reductions of X2 / X3 produce (sizes the partial arrays).
int x2_blocks(const Geo &g);
template <typename T> int x2_nblocks(const Geo &g);   // most partials a launch_x2<T> can write
int x3_blocks(const Geo &g);
template <typename T> int x3_nparts(const Geo &g);   // partials written by launch_x3<T> (all species)

// Reduction of the partials into state slots (single block, fixed order).
// A non-finite evaluation stores +inf in its slots (the line search then rejects it).
void launch_finalize(const RedBufs &r, int nf, int nm, double *fslot, double *mslot, DevState *st,
                     int count_kind, const int *gate, hipStream_t s, int nprob = 1, long long pstride = 0);

// Control kernels of the line search (one thread per problem of a batch).
enum CtlOp { CTL_BEGIN = 0, CTL_AMAX = 1, CTL_B = 2, CTL_FIT = 3, CTL_ACCEPT = 4, CTL_END = 5, CTL_PRIME = 6 };
void launch_ctl(DevState *st, int op, hipStream_t s, int nprob = 1, long long pstride = 0);

// Setup helpers: base_k = mu_k - beta V_k - z_k phi_fixed (-inf where V = +inf), and
// per-block counts of fluid nodes.
void launch_make_base(const Consts *cs, int S, long long N, const double *vext, const double *phi_fixed,
                      double *base, const double *mu_host, const double *z_host, double *count_part, int nblk,
                      hipStream_t s);
void launch_sum_to(const double *part, int n, double *dst, hipStream_t s);
// Line-search state records: nrec copies between strided places (byte strides), and the
// refresh gate of each record set from gates[i] (device ints).
void launch_copy_states(void *dst, long long dst_stride, const void *src, long long src_stride, int nrec,
                        hipStream_t s);
void launch_set_gates(DevState *first, long long stride, int nrec, const int *gates, hipStream_t s);
// dst <- the current iterate's density (role *sel) of every problem (gated as launch_copy).
void launch_copy_current(double *dst, const Roles &roles, long long count, hipStream_t s, int nprob,
                         long long pstride, const int *gate);
void launch_copy(double *dst, const double *src, long long count, hipStream_t s, int nprob = 1,
                 long long pstride = 0, const int *gate = nullptr);

}  // namespace dft
