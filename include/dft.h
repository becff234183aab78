/*
 * dft.h -- C ABI of the MI355X FFT/Picard solver for three-dimensional classical
 * density functional theory of charged hard spheres (Knepley, Karpeev, Davidovits,
 * Eisenberg, Gillespie: "An Efficient Algorithm for Classical Density Functional
 * Theory in Three Dimensions: Ionic Solutions").
 *
 * The library solves the Euler-Lagrange fixed point of the theory section,
 *     rho_i(x) = rho_i^bath exp(beta mu_i^HS,bath - beta V_i(x) + E_i[rho](x)),
 *     E_i = c_HS,i - beta mu_SC,i' - z_i beta e phi      (eqs. rhoEquation, excessChemicalPotential)
 * on a periodic uniform grid.  c_HS comes from fundamental measure theory
 * (eqs. nDef, omegaDef, muHS, Phi, conv; Appendix B spectra), the screening term from
 * the bulk-fluid expansion (eqs. muESexpansion, CplusPsiFunc, CplusPsiHat) and phi
 * from the finite-difference Poisson equation solved in Fourier space
 * (eqs. Poisson, potentialSolution, potentialConstraint).  Iteration: Picard with a
 * quadratic line search and the n3 <= 0.9 bound (nonlinear-solver section).
 *
 * Conventions
 *   - Grid: n[3] = (nx, ny, nz) nodes, spacings h[3]; node (ix, iy, iz) sits at
 *     (ix hx, iy hy, iz hz); the box is periodic with period n_d h_d.  Each n_d is
 *     1 or 2^a 3^b with 2 <= n_d <= 1024.
 *   - Fields are float64, laid out [species][z][y][x] (x fastest), and live in device
 *     (HIP) memory owned by the caller.  Scalars marked "host" are host memory.
 *   - Units: one caller length unit for h, radii and l_B; densities in unit^-3;
 *     energies in kT (beta-scaled); charge densities in e per unit^3.
 *   - Weighted densities are stacked as n0, n1, n2, n3, nV1(x,y,z), nV2(x,y,z).
 *   - Every call returns a dft_status; nothing throws or aborts across the ABI.
 *     Arguments are validated on the host before any HIP call, so the error paths
 *     run without a GPU.  dft_last_error() gives a thread-local message.
 *   - Work is enqueued on the stream given to dft_setup (dft_set_stream changes it).
 *     Functions that return host scalars synchronize that stream.
 *   - Ownership: the caller owns every device buffer (densities, potentials,
 *     workspace, outputs); the library owns only the opaque host dft_ctx and the HIP
 *     graph it captures.  dft_destroy never frees caller memory.
 *   - Thread safety: one ctx per stream; distinct ctxs are independent.
 */
#ifndef DFT_H
#define DFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DFT_MAX_SPECIES 8
#define DFT_NALPHA 10
#define DFT_MAX_N 1024

typedef struct dft_ctx dft_ctx;

typedef enum dft_status {
    DFT_OK = 0,
    DFT_E_INVALID_ARG = 1,      /* null pointer, non-positive h or R, negative density, bad flag */
    DFT_E_UNSUPPORTED_SIZE = 2, /* n_d not 1 or 2^a 3^b in [2, 1024], or too many species */
    DFT_E_WORKSPACE = 3,        /* workspace missing or smaller than dft_workspace_size */
    DFT_E_DEVICE = 4,           /* a HIP call failed */
    DFT_E_NONFINITE = 5,        /* a non-finite value appeared in G or in the norms */
    DFT_E_PACKING = 6,          /* max n3 >= eta_cap at the current iterate */
    DFT_E_NOT_CONVERGED = 7,    /* max_iter reached with r > tol */
    DFT_E_NOT_NEUTRAL = 8       /* bulk sum_k z_k rho_k not zero with electrostatics on */
} dft_status;

typedef enum dft_precision {
    DFT_FP64 = 0,       /* every transform and product in float64 */
    DFT_FP32_MIXED = 1  /* float32 transforms of differences from an FP64 reference state;
                           FP64 pointwise FMT, exponent, norms and master density */
} dft_precision;

/*
 * Hard-sphere free-energy density Phi (hard-sphere section: the scheme does not depend on
 * which fundamental-measure functional is used).  Every choice keeps the first two terms of
 * eq. (Phi); the third term and the bath (Appendix A) are:
 *   DFT_HS_RSLT        n2^3 (1 - xi^2)^3 / (24 pi (1 - n3)^2), as eq. (Phi) prints it;
 *                      Percus-Yevick bath (eqs. muHSBath, HSPressure).
 *   DFT_HS_ROSENFELD   (n2^3 - 3 n2 nV2.nV2) / (24 pi (1 - n3)^2), Rosenfeld's original
 *                      vector form; the same Percus-Yevick bath (vectors vanish in bulk).
 *   DFT_HS_WHITE_BEAR  (n2^3 - 3 n2 nV2.nV2) f(n3) / (36 pi),
 *                      f = (n3 + (1 - n3)^2 ln(1 - n3)) / (n3^2 (1 - n3)^2) (White Bear);
 *                      Boublik-Mansoori-Carnahan-Starling-Leland (BMCSL) bath.
 * The bound |nV2| <= n2 of Appendix C applies to all three (xi^2 <- min(xi^2, 1)).
 */
typedef enum dft_hs_functional {
    DFT_HS_RSLT = 0,
    DFT_HS_ROSENFELD = 1,
    DFT_HS_WHITE_BEAR = 2
} dft_hs_functional;

/* Flags for dft_params.flags */
#define DFT_FLAG_ALLOW_NON_NEUTRAL 1   /* accept a non-neutral bulk (finite-difference probes) */
#define DFT_FLAG_CUTOFF_LAMBDA     2   /* cut the screening kernel at lambda_i + lambda_j, not R_i + R_j */
#define DFT_FLAG_NO_AUTOTUNE       4   /* skip the launch-shape autotuner at setup (default shapes) */

/*
 * Problem statement (theory section; Appendix A for the bath).  Inline arrays keep
 * the struct self-contained for foreign-function callers.
 */
typedef struct dft_params {
    int32_t n[3];                         /* nodes along x, y, z */
    double h[3];                          /* grid spacings, > 0 */
    int32_t nspecies;                     /* 1 .. DFT_MAX_SPECIES */
    double radius[DFT_MAX_SPECIES];       /* R_k = sigma_k / 2, > 0 */
    double valence[DFT_MAX_SPECIES];      /* z_k */
    double rho_bulk[DFT_MAX_SPECIES];     /* rho_k^bath >= 0, unit^-3 */
    double bjerrum_length;                /* l_B = e^2 / (4 pi eps0 eps_r kT) in the length unit */
    int32_t electrostatics;               /* 0: hard spheres only; 1: bulk-fluid screening + Poisson */
    int32_t precision;                    /* dft_precision */
    double eta_cap;                       /* bound on max n3 in the line search; 0 selects 0.9 */
    int32_t flags;                        /* DFT_FLAG_* */
    int32_t hs_functional;                /* dft_hs_functional; 0 = eq. (Phi) as printed */
} dft_params;

/* Bath quantities of Appendix A, computed on the host in FP64. */
typedef struct dft_bulk_info {
    double mu_hs[DFT_MAX_SPECIES];   /* beta mu_k^HS,bath (eq. muHSBath; BMCSL for White Bear) */
    double beta_p;                   /* beta P^HS_bath (eq. HSPressure; BMCSL for White Bear) */
    double xi[4];                    /* xi_0 .. xi_3 */
    double gamma;                    /* MSA Gamma (eq. Gamma), 0 without electrostatics */
    double eta_msa;                  /* MSA eta at Gamma */
    double omega;                    /* MSA Omega at Gamma */
    double lambda[DFT_MAX_SPECIES];  /* lambda_k = R_k + 1/(2 Gamma) (bulk-fluid section) */
    double mu_es[DFT_MAX_SPECIES];   /* beta mu_k^ES,bath (reporting only; cancels in G) */
} dft_bulk_info;

/* Counters kept by a ctx since dft_setup or the last dft_solve start. */
typedef struct dft_stats {
    int64_t iterations;      /* accepted Picard steps */
    int64_t rejected;        /* line-search steps that did not lower the residual */
    int64_t g_evals;         /* full residual evaluations */
    int64_t n3_evals;        /* n3-only evaluations (step-cap path of the line search) */
    int64_t fp64_refresh;    /* FP64 reference evaluations (FP32-mixed only; counted since dft_setup) */
    double residual;         /* r at the current iterate */
    double alpha;            /* last accepted step */
    double max_n3;           /* max n3 at the current iterate */
    double step_cap;         /* current line-search step cap */
    int32_t compact_layout;  /* 1: the weighted densities pass from the z to the y transform
                                as 7 half spectra and from the y to the x transform as 9, and
                                their derivatives from the y to the z transform as 8 (the x
                                and y components of a vector density are -i k_x, -i k_y times
                                one field along a z pencil); 0: as 10 each; fixed at setup
                                (every pass on a compiled-length kernel) */
} dft_stats;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *dft_last_error(void);

/*
 * Bath thermodynamics (Appendix A: eqs. muHSBath, HSPressure, Gamma) on the host.
 * params: host, validated as in dft_setup.  out: host.  No GPU needed.
 */
dft_status dft_bulk(const dft_params *params, dft_bulk_info *out);

/*
 * Bytes of device workspace dft_setup needs for these parameters.  Host only.
 */
dft_status dft_workspace_size(const dft_params *params, size_t *bytes);

/*
 * Setup work done once per problem (discretization section: the bath and external
 * potentials are computed once): validates the parameters, solves the bath (Appendix A),
 * builds FFT plans and twiddle tables, and forms per species the fixed exponent
 *     beta mu_k^HS,bath - beta V_k(x) - z_k beta e phi_fixed(x)
 * (fixed charges enter the Poisson source only).
 *   beta_vext     device [S][nz][ny][nx] float64: beta V_k; +inf marks an excluded centre.
 *                 NULL means V = 0 everywhere.  Read during the call only.
 *   fixed_charge  device [nz][ny][nx] float64, e / unit^3; NULL means none.  Read only.
 *   workspace     device memory of at least dft_workspace_size bytes, 256-byte aligned,
 *                 owned by the caller and used by the ctx until dft_destroy.
 *   stream        hipStream_t as void* (NULL = default stream).
 *   out           receives the new ctx (host).
 * Errors: DFT_E_INVALID_ARG, DFT_E_UNSUPPORTED_SIZE, DFT_E_NOT_NEUTRAL, DFT_E_WORKSPACE
 * before any HIP call; DFT_E_INVALID_ARG also when beta_vext excludes every centre of every
 * species (no fluid node); DFT_E_DEVICE if a HIP call fails.
 */
dft_status dft_setup(const dft_params *params, const double *beta_vext, const double *fixed_charge,
                     void *workspace, size_t ws_bytes, void *stream, dft_ctx **out);

/* Change the stream subsequent calls enqueue on. */
dft_status dft_set_stream(dft_ctx *ctx, void *stream);

/*
 * One residual evaluation (eq. rhoEquation with eqs. conv, Phi, muHS, potentialSolution,
 * muESexpansion): G(rho) and the norm r = sqrt(sum_k sum_fluid ((rho_k - G_k)/rho_k^b)^2 / N_fluid).
 *   rho       device [S][N] float64 (read).
 *   g_out     device [S][N] float64 (written; NULL to skip).
 *   norm_out  host double (NULL to skip); if given, the stream is synchronized.
 * Uses the ctx's precision: in FP32-mixed mode the FP32 transforms act on rho - rho_ref
 * around the ctx's current reference state (set by dft_set_reference or dft_solve).
 * A non-finite evaluation (n3 >= 1 somewhere, or a non-finite rho) returns DFT_OK with
 * r = +inf; G is then not finite where the evaluation broke down.
 */
dft_status dft_residual(dft_ctx *ctx, const double *rho, double *g_out, double *norm_out);

/*
 * The intermediate fields of one FP64 residual evaluation at rho, for inspection and
 * parity tests (any output may be NULL):
 *   n_out     device [10][N]: weighted densities n_alpha (eq. nDef via eq. conv)
 *   dphi_out  device [10][N]: dPhi/dn_alpha (eq. Phi)
 *   c_out     device [S][N]:  E_k = c_HS,k + c_SC,k - z_k beta e phi (the exponent's rho-dependent part)
 *   phi_out   device [N]:     beta e phi from ions and fixed charges (eq. potentialSolution)
 */
dft_status dft_operators(dft_ctx *ctx, const double *rho, double *n_out, double *dphi_out,
                         double *c_out, double *phi_out);

/*
 * FP32-mixed only: make rho the reference state (one FP64 evaluation at rho).  Later
 * FP32 transforms act on differences from it.  No-op in FP64 mode.
 */
dft_status dft_set_reference(dft_ctx *ctx, const double *rho);

/*
 * One line-search Picard step (nonlinear-solver section) on rho_inout (device [S][N]),
 * updated in place.  alpha_out: accepted step (0 if the step was rejected), host.
 * norm_out: r at the new iterate, host.  Either may be NULL; the stream is synchronized.
 * Consecutive calls with the same buffer reuse the Picard image of the previous step.
 */
dft_status dft_picard_step(dft_ctx *ctx, double *rho_inout, double *alpha_out, double *norm_out);

/*
 * Picard iteration until r <= tol or max_iter accepted steps, starting from rho_inout
 * (device [S][N]) and leaving the last iterate there.  The step is a captured HIP graph
 * launched in chunks; the host reads the status between chunks.  In FP32-mixed mode the
 * FP64 reference is refreshed as the residual falls, and convergence is confirmed with
 * an FP64 evaluation.  iters_out, norm_out: host, may be NULL.
 * Returns DFT_E_NOT_CONVERGED, DFT_E_NONFINITE or DFT_E_PACKING on failure, leaving the
 * last finite iterate in rho_inout.
 */
dft_status dft_solve(dft_ctx *ctx, double *rho_inout, double tol, int32_t max_iter,
                     int32_t *iters_out, double *norm_out);

/*
 * Exactly nsteps line-search Picard steps (nonlinear-solver section) on rho_inout
 * (device [S][N]), launched as the captured HIP graph with no convergence stop and one
 * synchronization at the end.  Continues from the previous dft_run / dft_picard_step /
 * dft_solve state when rho_inout is the buffer those calls last used.  FP32-mixed mode
 * keeps the current reference state (no refresh).  iters_out (accepted steps) and
 * norm_out (r at the last iterate): host, may be NULL.  For benchmarks and for callers
 * that schedule their own stopping rule.
 */
dft_status dft_run(dft_ctx *ctx, double *rho_inout, int32_t nsteps, int32_t *iters_out, double *norm_out);

/* Passes of one residual evaluation, in launch order (see dft_profile). */
#define DFT_NPASS 10   /* x fwd, y fwd, z weights, y inv, x FMT, y fwd, z back+ES, y inv, x EL, reduce */

/*
 * Timing of the passes of one residual evaluation at rho (device [S][N]) in the ctx's
 * precision, measured with HIP events recorded between the launches on the ctx stream
 * and averaged over reps evaluations.  ms_out: host [DFT_NPASS], milliseconds per launch.
 */
dft_status dft_profile(dft_ctx *ctx, const double *rho, int32_t reps, double *ms_out);

/*
 * Bytes of device workspace dft_adjoint needs for these parameters.  Host only.
 */
dft_status dft_adjoint_workspace_size(const dft_params *params, size_t *bytes);

/*
 * Gradient of an observable O(rho*) through the converged fixed point rho* = G(rho*)
 * (eq. rhoEquation) by the implicit adjoint: with J = dG/drho = diag(G) H and H = dE/drho
 * symmetric, the adjoint weights w = G o lambda solve (diag(G)^-1 - H) w = dO/drho on
 * fluid nodes, by conjugate gradients preconditioned with diag(G) (a Krylov-accelerated
 * adjoint Picard iteration w <- G o (dO/drho + H w)).  Each iteration applies H through the
 * residual passes in FP64 with the exact Hessian of eq. (Phi).  Then
 *   dO/d(beta V_k(x)) = -w_k(x),
 *   dO/d rho_bulk_k, dO/d sigma_k = sum_i <w_i, d ln G_i / d theta>, including the bath terms
 *   of Appendix A (beta mu^HS, Gamma) and the screening kernel's dependence on R and Gamma;
 *   hard-core exclusion masks are held fixed.
 *   rho_star      device [S][N]: a converged solution (e.g. from dft_solve).
 *   dO_drho       device [S][N]: the observable's derivative.
 *   adj_ws        device workspace of dft_adjoint_workspace_size bytes, 256-byte aligned.
 *   tol           relative residual of the adjoint system; max_iter its iteration limit.
 *   dO_dvext      device [S][N] out (NULL to skip); dO_drho_bulk, dO_dsigma: host [S] out (NULL to skip).
 *   iters_out, resid_out: host, may be NULL.  Synchronizes the stream.
 * Supports up to 4 species and n_x <= 384.  Errors: DFT_E_NOT_CONVERGED, DFT_E_NONFINITE
 * (the system is not positive definite at rho*: rho* is not a stable solution).
 */
dft_status dft_adjoint(dft_ctx *ctx, const double *rho_star, const double *dO_drho, void *adj_ws, size_t adj_ws_bytes,
                       double tol, int32_t max_iter, double *dO_dvext, double *dO_drho_bulk, double *dO_dsigma,
                       int32_t *iters_out, double *resid_out);

/*
 * dft_adjoint without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  The same
 * computation and results as dft_adjoint; the workspace is a fixed array of
 * DFT_ADJOINT_NOALLOC_MAX_BYTES in the library's device image, one per GPU, held until the
 * process ends.  The call allocates no device or host memory (an error message is formatted
 * only on failure) and needs dft_adjoint_workspace_size(params) <= DFT_ADJOINT_NOALLOC_MAX_BYTES
 * (about a 40^3 grid with three species), else DFT_E_WORKSPACE.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (several threads, or streams not ordered
 * against each other) race and must be serialized by the caller.  Nothing in the array needs
 * to start at zero; the previous call's contents are overwritten.  Call with the ctx's device
 * current.  Arguments, outputs and errors otherwise as dft_adjoint.
 */
#define DFT_ADJOINT_NOALLOC_MAX_BYTES (64u << 20)
dft_status dft_adjoint_noalloc(dft_ctx *ctx, const double *rho_star, const double *dO_drho, double tol,
                               int32_t max_iter, double *dO_dvext, double *dO_drho_bulk, double *dO_dsigma,
                               int32_t *iters_out, double *resid_out);

/*
 * Newton-Krylov solve of the fixed point rho = G(rho) (eq. rhoEquation), an alternative to
 * the Picard iteration of the nonlinear-solver section with the exact Jacobian instead of a
 * finite-difference one: each step solves (I - diag(G) H) d = G - rho, symmetrized as
 * (diag(G)^-1 - H) d = (G - rho) / G on fluid nodes, by conjugate gradients preconditioned
 * with diag(G) and started from the Picard direction G - rho, with H applied through the
 * FP64 residual passes and the exact FMT Hessian (as dft_adjoint); the forcing term shrinks
 * with the residual.  The step is limited to keep every density positive and backtracked
 * until the residual norm decreases and max n3 stays below eta_cap.
 *   rho           device [S][N], in: start, out: the last accepted iterate.
 *   adj_ws        device workspace of dft_adjoint_workspace_size bytes, 256-byte aligned.
 *   tol           residual target (the same norm as dft_solve); max_iter Newton steps.
 *   iters_out, cg_iters_out, norm_out: host, may be NULL.  FP64 evaluations in any precision.
 * Same limits as dft_adjoint (S <= 4, n_x <= 384).  Errors: DFT_E_NOT_CONVERGED (max_iter or
 * no decrease along the step), DFT_E_NONFINITE, DFT_E_PACKING.
 */
dft_status dft_newton(dft_ctx *ctx, double *rho, void *adj_ws, size_t adj_ws_bytes, double tol, int32_t max_iter,
                      int32_t *iters_out, int32_t *cg_iters_out, double *norm_out);

/*
 * Screening operator of the reference-fluid-density (RFD) electrostatics (RFD section, eqs.
 * rhoRef, rhoRefKDotProduct, screening-kernel-hat): each of the ctx's S fields f_i is averaged
 * over the ball of radius R_SC(x) centred on every grid point x,
 *   f_ref_i(x) = N^-1 sum_k f_hat_i(k) B(|k| R_SC(x)) exp(i k.x),  B(t) = 3 (sin t - t cos t) / t^3,
 * on the k set of eq. Kvalues (f_hat: forward DFT).  The paper evaluates this as an O(N^2) dot
 * product per grid point.  Here B is interpolated in the radius: the fields are convolved by FFT
 * with the balls of `nodes` first-kind Chebyshev radii spanning [min R_SC, max R_SC], and each
 * point combines the results with the barycentric Lagrange weights of its own R_SC.  Cost: one
 * forward and `nodes` inverse 3-D transforms per field.  The error falls geometrically once
 * `nodes` exceeds about k_max (max R_SC - min R_SC) / 2 (k_max the largest |k| of the grid); a
 * constant R_SC is exact with any `nodes` (one convolution).
 *   f      device [S][N] FP64 (pass alpha_i rho_i for the weighted average of eq. rhoBarDef).
 *   rsc    device [N] FP64, R_SC(x) in the length unit, positive and finite.
 *   nodes  1 .. DFT_RFD_MAX_NODES.
 *   f_ref  device [S][N] FP64 out; may be the same buffer as f.
 * FP64 in either precision.  Uses the ctx's spectral buffers and the line-search buffers that do
 * not hold the current iterate (the iterate, its G and the captured step are kept); reads the
 * line-search state and the R_SC range back to the host, so it synchronizes the ctx stream.
 * Errors: DFT_E_INVALID_ARG (NULL pointers, nodes out of range, an R_SC that is not positive and
 * finite, a batch group ctx).
 */
#define DFT_RFD_MAX_NODES 128
dft_status dft_rfd_reference(dft_ctx *ctx, const double *f, const double *rsc, int32_t nodes, double *f_ref);

/*
 * Batches of independent state points (different concentrations, valences, radii, grids).
 * Points of one shape (n, nspecies, precision) form a group; every pass of a residual
 * evaluation is ONE launch over all points of a group, the line-search state machines run
 * one device thread per point, and a whole Picard step of a group is one captured HIP
 * graph.  Converged points retire (their work is gated off) while the others continue.
 */
typedef struct dft_batch dft_batch;

/* Bytes of device workspace for `count` state points.  Host only. */
dft_status dft_batch_workspace_size(const dft_params *params, int32_t count, size_t *bytes);

/*
 * Set up `count` state points.  params: host [count].  beta_vext, fixed_charge: host arrays
 * [count] of device pointers (each as in dft_setup; the arrays themselves may be NULL).
 * workspace: device, dft_batch_workspace_size bytes, 256-byte aligned, caller-owned.
 */
dft_status dft_setup_batch(const dft_params *params, int32_t count, const double *const *beta_vext,
                           const double *const *fixed_charge, void *workspace, size_t ws_bytes, void *stream,
                           dft_batch **out);

/* The per-point ctx (for dft_residual, dft_get_stats, dft_adjoint ...); owned by the batch. */
dft_status dft_batch_member(dft_batch *batch, int32_t i, dft_ctx **out);

/*
 * Solve every state point (as dft_solve) from the densities rho_inout[i] (host array of
 * device pointers).  iters_out, norm_out, status_out: host [count], may be NULL.  Returns
 * the first failing point's status (DFT_OK if all converged).
 */
dft_status dft_solve_batch(dft_batch *batch, double *const *rho_inout, double tol, int32_t max_iter,
                           int32_t *iters_out, double *norm_out, int32_t *status_out);

/* Free the batch, its points' ctxs and graphs; caller memory is untouched. */
dft_status dft_batch_destroy(dft_batch *batch);

/* Counters of the ctx (host out). */
dft_status dft_get_stats(dft_ctx *ctx, dft_stats *out);

/*
 * Launch shapes of the FFT pass kernels (batched FFT schedules, Section 4's many
 * transforms per step): for each tunable pass and each transform precision {FP64, FP32},
 * the index of the tile shape in use, as DFT_SCHEDULE_LEN int32 laid out [pass][precision].
 * Passes, in order: 0 the inverse y pass of the ten weighted-density spectra, 1 the plain z
 * pass, 2 the z pass of the weighted densities (Z1), 3 the z back-convolution (Z2), 4 the
 * forward y pass of the ten derivative spectra, 5 the y passes of the species spectra.
 * y passes and plain z: 10 shapes (five tile widths / thread counts with two LDS buffers,
 * then the same five with one); Z1: 6 (three tile widths fused with the forward z transform
 * of the species, then the same widths after a separate plain z pass); Z2: 3.  dft_setup
 * picks them by timing every shape on the device (the autotuner; DFT_FLAG_NO_AUTOTUNE keeps
 * shape 0).  Every shape of a pass performs the same arithmetic in the same order, so the
 * shapes change run time only, never results.  dft_set_schedule validates each index
 * (DFT_E_INVALID_ARG if out of range) and drops the ctx's captured step graph.
 */
#define DFT_TUNE_PASSES 6
#define DFT_SCHEDULE_LEN (2 * DFT_TUNE_PASSES)
dft_status dft_get_schedule(const dft_ctx *ctx, int32_t *shapes_out);
dft_status dft_set_schedule(dft_ctx *ctx, const int32_t *shapes);

/* Free the ctx and its graph; caller memory is untouched.  NULL is accepted. */
dft_status dft_destroy(dft_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DFT_H */
