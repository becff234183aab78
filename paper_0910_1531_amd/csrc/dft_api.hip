// C ABI of the solver (include/dft.h): context, workspace layout, the residual
// evaluation sequence, the device-controlled line-search step, HIP graph capture and
// the solve loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "dft_adjoint.h"
#include "dft_host.h"
#include "dft_kernels.h"
#include "dft_screen.h"
#include "dft_tune.h"

using namespace dft;

namespace {

thread_local std::string g_last_error;

dft_status fail(dft_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) throw HipError(std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ workspace layout
struct Layout {
    size_t consts, state, tw64[3], tw32[3], fpart, mpart, fflag, mflag, specA, specB;
    size_t base, rho0, g0, ga, gb, gs, rho_t, rho_t2, rho_t3, rho_ref, lp, nref, phi_fix, count_part;
    size_t tab64;
    int ntab;
    size_t total;
    int red_cap;
    int count_blocks;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout make_layout(const dft_params *p) {
    Layout L;
    const long long N = (long long)p->n[0] * p->n[1] * p->n[2];
    const long long Kx = p->n[0] / 2 + 1;
    const long long NC = Kx * p->n[1] * p->n[2];
    const int S = p->nspecies;
    Geo g{};
    g.nx = p->n[0];
    g.ny = p->n[1];
    g.nz = p->n[2];
    g.S = S;
    L.red_cap = std::max(x2_blocks(g), x3_blocks(g)) + 16;
    L.count_blocks = (int)std::min<long long>((S * N + 255) / 256, 4096);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.consts = take(sizeof(Consts));
    L.state = take(sizeof(DevState));
    for (int d = 0; d < 3; ++d) {
        L.tw64[d] = take(2 * sizeof(double) * p->n[d]);
        L.tw32[d] = take(2 * sizeof(float) * p->n[d]);
    }
    L.fpart = take(sizeof(double) * L.red_cap);
    L.mpart = take(sizeof(double) * L.red_cap);
    L.fflag = take(sizeof(int) * L.red_cap);
    L.mflag = take(sizeof(int) * L.red_cap);
    L.count_part = take(sizeof(double) * L.count_blocks);
    L.specA = take(2 * sizeof(double) * NC * S);
    L.specB = take(2 * sizeof(double) * NC * DFT_NALPHA);
    const size_t F = sizeof(double) * (size_t)N * S;
    L.base = take(F);
    L.rho0 = take(F);
    L.g0 = take(F);
    L.ga = take(F);
    L.gb = take(F);
    L.gs = take(F);
    L.rho_t = take(F);
    L.rho_t2 = take(F);
    L.rho_t3 = take(F);
    L.phi_fix = take(sizeof(double) * (size_t)N);
    if (p->precision == DFT_FP32_MIXED) {
        L.rho_ref = take(F);
        L.lp = take(F);
        L.nref = take(sizeof(float) * (size_t)N * DFT_NALPHA);
    } else {
        L.rho_ref = L.lp = L.nref = 0;
    }
    L.ntab = spec_table_rows(p->n[2], S, p->electrostatics ? 1 : 0);
    L.tab64 = L.ntab ? take(sizeof(double) * (size_t)NC * L.ntab) : 0;
    L.total = off;
    return L;
}

}  // namespace

struct dft_ctx {
    dft_params p;
    dft_bulk_info bulk;
    Consts hc;
    Layout lay;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    Geo geo{};
    Consts *cs = nullptr;
    DevState *st = nullptr;
    void *specA = nullptr, *specB = nullptr;
    double *base = nullptr, *rho0 = nullptr, *g0 = nullptr, *ga = nullptr, *gb = nullptr, *gs = nullptr;
    double *rho_t = nullptr, *rho_ref = nullptr, *lp = nullptr, *phi_fix = nullptr;
    float *nref = nullptr;
    // line-search buffers by role: densities {rho0, rho_t, rho_t2, rho_t3}, images {g0, gb, ga, gs};
    // the state's sel names the current iterate's (role 0 after a fresh state)
    Roles roles{};
    RedBufs red{};
    int nf_parts = 0, nm_parts = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *step_rho = nullptr;   // caller buffer whose iterate the current role holds
    long long refreshes = 0;
    bool mixed = false;
};

namespace {

// Options of one residual evaluation.
struct Eval {
    bool trial = false;            // rho_t = rho0 + alpha (g0 - rho0)
    int kind = -1;                 // >= 0: a line-search pass on the rotating buffers (RoleKind);
                                   // src, g0, rho_t and g_out then come from the roles
    const double *src = nullptr;   // plain: rho; trial: rho0
    const double *g0 = nullptr;
    const double *alpha = nullptr;
    double *g_out = nullptr;
    double *e_out = nullptr;
    double *n_out = nullptr;
    double *dphi_out = nullptr;
    double *fslot = nullptr;
    double *mslot = nullptr;
    int count_kind = 1;
    const int *gate = nullptr;
    bool fp64 = true;              // transforms in FP64 (FP64 ctx, or FP32-mixed refresh/inspection)
    bool refresh = false;          // FP32-mixed: write the reference fields
    hipEvent_t *events = nullptr;  // if set: DFT_NPASS + 1 events recorded around the launches
};

inline void mark(const Eval &ev, int k, hipStream_t s) {
    if (ev.events) HIPCHK(hipEventRecord(ev.events[k], s));
}

template <typename T>
void enqueue_eval_t(dft_ctx *c, const Eval &ev, hipStream_t s) {
    const Geo &g = c->geo;
    const bool diff = c->mixed && !ev.fp64;
    const double *rho_eval = ev.trial ? c->rho_t : ev.src;
    XFwdArgs xa{};
    xa.src = ev.src;
    xa.g0 = ev.g0;
    xa.alpha = ev.alpha;
    xa.rho_t = ev.trial ? c->rho_t : nullptr;
    xa.ref = diff ? c->rho_ref : nullptr;
    xa.spec = c->specA;
    xa.nfield = g.S;
    xa.mode = ev.trial ? XF_TRIAL : XF_PLAIN;
    xa.gate = ev.gate;
    if (ev.kind >= 0) {
        xa.roles = c->roles;
        xa.kind = ev.kind;
    }
    mark(ev, 0, s);
    launch_x_forward<T>(g, xa, s);
    mark(ev, 1, s);
    YArgs ya{c->specA, g.S, -1, ev.gate};
    launch_y<T>(g, ya, s);
    mark(ev, 2, s);
    Z1Args z1{c->specA, c->specB, 0, diff ? 1 : 0, ev.gate};
    launch_z1<T>(g, z1, s);
    mark(ev, 3, s);
    YArgs yb{c->specB, DFT_NALPHA, 1, ev.gate};
    yb.vec = g.compact ? 1 : 0;
    launch_y<T>(g, yb, s);
    mark(ev, 4, s);
    X2Args x2{};
    x2.specB = c->specB;
    x2.hs = c->p.hs_functional;
    x2.mode = X2_FULL;
    x2.nref = diff ? c->nref : nullptr;
    x2.nref_out = ev.refresh ? c->nref : nullptr;
    x2.n_out = ev.n_out;
    x2.dphi_out = ev.dphi_out;
    x2.red = c->red;
    x2.gate = ev.gate;
    const int nb2 = launch_x2<T>(g, x2, s);
    mark(ev, 5, s);
    YArgs yc{c->specB, DFT_NALPHA, -1, ev.gate};
    yc.vec = g.compact ? 2 : 0;
    launch_y<T>(g, yc, s);
    mark(ev, 6, s);
    Z2Args z2{};
    z2.specB = c->specB;
    z2.specA = c->specA;
    z2.mode = Z2_EL;
    z2.gate = ev.gate;
    launch_z2<T>(g, z2, s);
    mark(ev, 7, s);
    YArgs yd{c->specA, g.S, 1, ev.gate};
    launch_y<T>(g, yd, s);
    mark(ev, 8, s);
    X3Args x3{};
    x3.specA = c->specA;
    x3.nfield = g.S;
    x3.raw = 0;
    x3.base = diff ? c->lp : c->base;
    x3.rho_t = rho_eval;
    x3.g_out = ev.g_out;
    x3.e_out = ev.e_out;
    x3.e_phi = (ev.e_out && c->p.electrostatics) ? c->phi_fix : nullptr;
    x3.lp_out = ev.refresh ? c->lp : nullptr;
    x3.red = c->red;
    x3.gate = ev.gate;
    if (ev.kind >= 0) {
        x3.roles = c->roles;
        x3.kind = ev.kind;
    }
    launch_x3<T>(g, x3, s);
    mark(ev, 9, s);
    launch_finalize(c->red, x3_nparts<T>(g), nb2, ev.fslot, ev.mslot, c->st,
                    ev.count_kind, ev.gate, s, g.nprob, g.pstride);
    mark(ev, 10, s);
}

void enqueue_eval(dft_ctx *c, const Eval &ev, hipStream_t s) {
    if (ev.fp64 || !c->mixed) enqueue_eval_t<double>(c, ev, s);
    else enqueue_eval_t<float>(c, ev, s);
}

// max n3 at rho0 + alpha (g0 - rho0) without the rest of G (linear in rho).
template <typename T>
void enqueue_n3_t(dft_ctx *c, const double *alpha, double *mslot, const int *gate, hipStream_t s) {
    const Geo &g = c->geo;
    const bool diff = c->mixed;
    XFwdArgs xa{};
    xa.alpha = alpha;
    xa.roles = c->roles;
    xa.kind = ROLE_N3;
    xa.ref = diff ? c->rho_ref : nullptr;
    xa.spec = c->specA;
    xa.nfield = g.S;
    xa.mode = XF_TRIAL;
    xa.gate = gate;
    launch_x_forward<T>(g, xa, s);
    YArgs ya{c->specA, g.S, -1, gate};
    launch_y<T>(g, ya, s);
    Z1Args z1{c->specA, c->specB, 1, diff ? 1 : 0, gate};
    launch_z1<T>(g, z1, s);
    YArgs yb{c->specB, 1, 1, gate};
    launch_y<T>(g, yb, s);
    X2Args x2{};
    x2.specB = c->specB;
    x2.hs = c->p.hs_functional;
    x2.mode = X2_N3_ONLY;
    x2.nref = diff ? c->nref : nullptr;
    x2.red = c->red;
    x2.gate = gate;
    const int nb2 = launch_x2<T>(g, x2, s);
    launch_finalize(c->red, 0, nb2, nullptr, mslot, c->st, 2, gate, s, g.nprob, g.pstride);
}

void enqueue_step(dft_ctx *c, hipStream_t s) {
    DevState *st = c->st;
    launch_ctl(st, CTL_BEGIN, s, c->geo.nprob, c->geo.pstride);
    Eval e1;
    e1.trial = true;
    e1.kind = ROLE_B;
    e1.alpha = &st->alpha_trial;
    e1.fslot = &st->f1;
    e1.mslot = &st->m1;
    e1.gate = &st->gate_full1;
    e1.fp64 = !c->mixed;
    enqueue_eval(c, e1, s);
    if (c->mixed) enqueue_n3_t<float>(c, &st->alpha_trial, &st->m1, &st->gate_part1, s);
    else enqueue_n3_t<double>(c, &st->alpha_trial, &st->m1, &st->gate_part1, s);
    launch_ctl(st, CTL_AMAX, s, c->geo.nprob, c->geo.pstride);
    Eval ea = e1;
    ea.kind = ROLE_A;
    ea.fslot = &st->fa;
    ea.mslot = &st->ma;
    ea.gate = &st->gate_a;
    enqueue_eval(c, ea, s);
    launch_ctl(st, CTL_B, s, c->geo.nprob, c->geo.pstride);
    Eval eb = e1;
    eb.kind = ROLE_B;
    eb.fslot = &st->fb;
    eb.mslot = &st->mb;
    eb.gate = &st->gate_b;
    enqueue_eval(c, eb, s);
    launch_ctl(st, CTL_FIT, s, c->geo.nprob, c->geo.pstride);
    Eval es = e1;
    es.kind = ROLE_S;
    es.fslot = &st->fs;
    es.mslot = &st->ms;
    es.gate = &st->gate_s;
    enqueue_eval(c, es, s);
    // acceptance rotates the roles: no arrays move
    launch_ctl(st, CTL_ACCEPT, s, c->geo.nprob, c->geo.pstride);
    launch_ctl(st, CTL_END, s, c->geo.nprob, c->geo.pstride);
}

// FP64 evaluation at rho0 that also becomes the FP32-mixed reference (or plain prime).
// With `gated`, only the problems of a batch whose gate_refresh is set take part.
void enqueue_prime(dft_ctx *c, hipStream_t s, bool gated = false) {
    DevState *st = c->st;
    const int *gate = gated ? &st->gate_refresh : nullptr;
    Eval e;
    e.gate = gate;
    e.trial = true;
    e.kind = ROLE_PRIME;   // the current iterate itself (alpha = 0), its image into its role
    e.alpha = &st->alpha_zero;
    e.fslot = &st->f0;
    e.mslot = &st->m0;
    e.fp64 = true;
    if (c->mixed) {
        launch_copy_current(c->rho_ref, c->roles, (long long)c->geo.S * c->geo.N, s, c->geo.nprob, c->geo.pstride,
                            gate);
        e.refresh = true;
    }
    enqueue_eval(c, e, s);
    launch_ctl(st, CTL_PRIME, s, c->geo.nprob, c->geo.pstride);
}

DevState read_state(dft_ctx *c) {
    DevState h;
    HIPCHK(hipMemcpyAsync(&h, c->st, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return h;
}

void write_state(dft_ctx *c, const DevState &h) {
    HIPCHK(hipMemcpyAsync(c->st, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
}

DevState fresh_state(dft_ctx *c, double tol, long long max_iter) {
    DevState h;
    std::memset(&h, 0, sizeof h);
    h.cap = 1.0;
    h.tol = tol;
    h.max_iter = max_iter;
    h.nfluid = c->hc.nfluid;
    h.eta_cap = c->hc.eta_cap;
    h.alpha_zero = 0.0;
    h.alpha_one = 1.0;
    h.gate_one = 1;
    return h;
}

void ensure_graph(dft_ctx *c) {
    if (c->gexec) return;
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_step(c, c->cap_stream);
    } catch (...) {
        hipGraph_t tmp;
        (void)hipStreamEndCapture(c->cap_stream, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
    }
    HIPCHK(hipStreamEndCapture(c->cap_stream, &c->graph));
    HIPCHK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
}

dft_status status_from(const DevState &h) {
    if (h.status == DFT_E_NONFINITE) return fail(DFT_E_NONFINITE, "non-finite residual at the current iterate");
    if (h.status == DFT_E_PACKING) return fail(DFT_E_PACKING, "max n3 reached the packing cap at the current iterate");
    return DFT_OK;
}

template <typename F>
dft_status guarded(F &&f) {
    try {
        return f();
    } catch (const HipError &e) {
        return fail(DFT_E_DEVICE, e.what());
    } catch (const std::exception &e) {
        return fail(DFT_E_DEVICE, e.what());
    }
}

}  // namespace

extern "C" {

const char *dft_last_error(void) { return g_last_error.c_str(); }

dft_status dft_bulk(const dft_params *params, dft_bulk_info *out) {
    std::string msg;
    dft_status st = bulk_info(params, out, &msg);
    if (st != DFT_OK) return fail(st, msg);
    return DFT_OK;
}

dft_status dft_workspace_size(const dft_params *params, size_t *bytes) {
    std::string msg;
    dft_status st = validate(params, &msg);
    if (st != DFT_OK) return fail(st, msg);
    if (!bytes) return fail(DFT_E_INVALID_ARG, "bytes is NULL");
    *bytes = make_layout(params).total;
    return DFT_OK;
}

dft_status dft_setup(const dft_params *params, const double *beta_vext, const double *fixed_charge, void *workspace,
                     size_t ws_bytes, void *stream, dft_ctx **out) {
    std::string msg;
    if (!out) return fail(DFT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    dft_bulk_info bi;
    dft_status st = bulk_info(params, &bi, &msg);
    if (st != DFT_OK) return fail(st, msg);
    Layout lay = make_layout(params);
    if (!workspace) return fail(DFT_E_WORKSPACE, "workspace is NULL");
    if (ws_bytes < lay.total) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, lay.total);
        return fail(DFT_E_WORKSPACE, buf);
    }
    if (((uintptr_t)workspace) % 256 != 0) return fail(DFT_E_WORKSPACE, "workspace must be 256-byte aligned");
    FftPlan plans[3];
    for (int d = 0; d < 3; ++d)
        if (!make_plan(params->n[d], &plans[d])) return fail(DFT_E_UNSUPPORTED_SIZE, "no FFT plan for this size");
    if (fixed_charge && !params->electrostatics)
        return fail(DFT_E_INVALID_ARG, "fixed_charge given with electrostatics off");

    dft_ctx *c = new dft_ctx();
    c->p = *params;
    c->bulk = bi;
    c->lay = lay;
    c->stream = (hipStream_t)stream;
    c->ws = (char *)workspace;
    c->mixed = params->precision == DFT_FP32_MIXED;
    fill_consts(params, bi, &c->hc);
    st = guarded([&]() -> dft_status {
        char *w = c->ws;
        c->cs = (Consts *)(w + lay.consts);
        c->st = (DevState *)(w + lay.state);
        c->specA = w + lay.specA;
        c->specB = w + lay.specB;
        c->base = (double *)(w + lay.base);
        c->rho0 = (double *)(w + lay.rho0);
        c->g0 = (double *)(w + lay.g0);
        c->ga = (double *)(w + lay.ga);
        c->gb = (double *)(w + lay.gb);
        c->gs = (double *)(w + lay.gs);
        c->rho_t = (double *)(w + lay.rho_t);
        c->roles.rho[0] = c->rho0;
        c->roles.rho[1] = c->rho_t;
        c->roles.rho[2] = (double *)(w + lay.rho_t2);
        c->roles.rho[3] = (double *)(w + lay.rho_t3);
        c->roles.G[0] = c->g0;
        c->roles.G[1] = c->gb;
        c->roles.G[2] = c->ga;
        c->roles.G[3] = c->gs;
        c->roles.sel = &c->st->sel;
        c->phi_fix = (double *)(w + lay.phi_fix);
        if (c->mixed) {
            c->rho_ref = (double *)(w + lay.rho_ref);
            c->lp = (double *)(w + lay.lp);
            c->nref = (float *)(w + lay.nref);
        }
        c->red.fpart = (double *)(w + lay.fpart);
        c->red.mpart = (double *)(w + lay.mpart);
        c->red.fflag = (int *)(w + lay.fflag);
        c->red.mflag = (int *)(w + lay.mflag);
        c->red.cap = lay.red_cap;
        Geo &g = c->geo;
        g.cs = c->cs;
        g.nx = params->n[0];
        g.ny = params->n[1];
        g.nz = params->n[2];
        g.Kx = c->hc.Kx;
        g.S = params->nspecies;
        g.es = c->hc.es;
        g.cut_lambda = c->hc.cut_lambda;
        g.N = c->hc.N;
        g.NC = c->hc.NC;
        DevPlan *dp[3] = {&g.px, &g.py, &g.pz};
        for (int d = 0; d < 3; ++d) {
            dp[d]->L = plans[d].L;
            dp[d]->nr = plans[d].nr;
            for (int k = 0; k < kMaxRadices; ++k) dp[d]->r[k] = plans[d].r[k];
            std::vector<double> tw;
            twiddles(params->n[d], &tw);
            std::vector<float> tf(tw.begin(), tw.end());
            HIPCHK(hipMemcpyAsync(w + lay.tw64[d], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(hipMemcpyAsync(w + lay.tw32[d], tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            g.tw64[d] = w + lay.tw64[d];
            g.tw32[d] = w + lay.tw32[d];
        }
        HIPCHK(hipMemcpyAsync(c->cs, &c->hc, sizeof(Consts), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (lay.ntab) {
            g.ntab = lay.ntab;
            g.tab64 = (const double *)(w + lay.tab64);
            launch_spec_tables(g, c->stream);
        }
        // compact vector layout when every pass of the evaluation runs a compiled-length kernel
        g.compact = (g.tab64 && x_ct_pairs(g.nx) > 0 && y_ct_variants(g.ny, false) > 0 &&
                     z_ct_variants(g.nz) > 0 && !(g.es && g.cut_lambda)) ? 1 : 0;
        if (!(params->flags & DFT_FLAG_NO_AUTOTUNE)) {
            TuneBufs tb{c->specA, 2 * sizeof(double) * (size_t)g.NC * g.S, c->specB,
                        2 * sizeof(double) * (size_t)g.NC * DFT_NALPHA};
            autotune(g, tb, true, c->mixed, c->stream);
        }
        // potential of the fixed charges (Poisson source only), FP64
        const double *phi = nullptr;
        if (fixed_charge && params->electrostatics) {
            XFwdArgs xa{};
            xa.src = fixed_charge;
            xa.spec = c->specA;
            xa.nfield = 1;
            xa.mode = XF_PLAIN;
            launch_x_forward<double>(g, xa, c->stream);
            YArgs ya{c->specA, 1, -1, nullptr};
            launch_y<double>(g, ya, c->stream);
            Z2Args z2{};
            z2.specA = c->specA;
            z2.mode = Z2_POISSON;
            z2.nsrc = 1;
            z2.wsrc[0] = 1.0;
            launch_z2<double>(g, z2, c->stream);
            YArgs yb{c->specA, 1, 1, nullptr};
            launch_y<double>(g, yb, c->stream);
            X3Args x3{};
            x3.specA = c->specA;
            x3.nfield = 1;
            x3.raw = 1;
            x3.raw_out = c->phi_fix;
            launch_x3<double>(g, x3, c->stream);
            phi = c->phi_fix;
        } else {
            HIPCHK(hipMemsetAsync(c->phi_fix, 0, sizeof(double) * g.N, c->stream));
        }
        double *cnt = (double *)(w + lay.count_part);
        launch_make_base(c->cs, g.S, g.N, beta_vext, phi, c->base, bi.mu_hs, params->valence, cnt, lay.count_blocks,
                         c->stream);
        double nfl = 0.0;
        launch_sum_to(cnt, lay.count_blocks, &c->st->nfluid, c->stream);
        HIPCHK(hipMemcpyAsync(&nfl, &c->st->nfluid, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (!(nfl > 0.0)) return fail(DFT_E_INVALID_ARG, "no fluid node: every centre is excluded");
        c->hc.nfluid = nfl;
        HIPCHK(hipMemcpyAsync(c->cs, &c->hc, sizeof(Consts), hipMemcpyHostToDevice, c->stream));
        DevState h = fresh_state(c, 0.0, 0);
        write_state(c, h);
        return DFT_OK;
    });
    if (st != DFT_OK) {
        delete c;
        return st;
    }
    *out = c;
    g_last_error.clear();
    return DFT_OK;
}

dft_status dft_set_stream(dft_ctx *ctx, void *stream) {
    if (!ctx) return fail(DFT_E_INVALID_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
    return DFT_OK;
}

dft_status dft_set_reference(dft_ctx *ctx, const double *rho) {
    if (!ctx || !rho) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    if (!ctx->mixed) return DFT_OK;
    return guarded([&]() -> dft_status {
        DevState h = read_state(ctx);
        h.tol = 0.0;
        h.sel = 0;
        write_state(ctx, h);
        launch_copy(ctx->rho0, rho, (long long)ctx->geo.S * ctx->geo.N, ctx->stream);
        enqueue_prime(ctx, ctx->stream);
        ctx->refreshes += 1;
        ctx->step_rho = nullptr;
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return DFT_OK;
    });
}

dft_status dft_residual(dft_ctx *ctx, const double *rho, double *g_out, double *norm_out) {
    if (!ctx || !rho) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    return guarded([&]() -> dft_status {
        if (ctx->mixed && ctx->refreshes == 0) {
            // no reference state yet: rho becomes the reference
            dft_status s2 = dft_set_reference(ctx, rho);
            if (s2 != DFT_OK) return s2;
        }
        Eval e;
        e.src = rho;
        e.g_out = g_out ? g_out : ctx->gs;
        e.fslot = &ctx->st->best_f;
        e.mslot = nullptr;
        e.fp64 = !ctx->mixed;
        enqueue_eval(ctx, e, ctx->stream);
        ctx->step_rho = nullptr;
        if (norm_out) {
            DevState h = read_state(ctx);
            *norm_out = std::sqrt(h.best_f / ctx->hc.nfluid);
        }
        return DFT_OK;
    });
}

dft_status dft_operators(dft_ctx *ctx, const double *rho, double *n_out, double *dphi_out, double *c_out,
                         double *phi_out) {
    if (!ctx || !rho) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    return guarded([&]() -> dft_status {
        Eval e;
        e.src = rho;
        e.g_out = ctx->gs;
        e.e_out = c_out;
        e.n_out = n_out;
        e.dphi_out = dphi_out;
        e.fslot = &ctx->st->best_f;
        e.fp64 = true;
        e.count_kind = 0;
        enqueue_eval(ctx, e, ctx->stream);
        if (phi_out) {
            const Geo &g = ctx->geo;
            if (!ctx->p.electrostatics) {
                HIPCHK(hipMemsetAsync(phi_out, 0, sizeof(double) * g.N, ctx->stream));
            } else {
                XFwdArgs xa{};
                xa.src = rho;
                xa.spec = ctx->specA;
                xa.nfield = g.S;
                xa.mode = XF_PLAIN;
                launch_x_forward<double>(g, xa, ctx->stream);
                YArgs ya{ctx->specA, g.S, -1, nullptr};
                launch_y<double>(g, ya, ctx->stream);
                Z2Args z2{};
                z2.specA = ctx->specA;
                z2.mode = Z2_POISSON;
                z2.nsrc = g.S;
                for (int i = 0; i < g.S; ++i) z2.wsrc[i] = ctx->p.valence[i];
                launch_z2<double>(g, z2, ctx->stream);
                YArgs yb{ctx->specA, 1, 1, nullptr};
                launch_y<double>(g, yb, ctx->stream);
                X3Args x3{};
                x3.specA = ctx->specA;
                x3.nfield = 1;
                x3.raw = 1;
                x3.addend = ctx->phi_fix;
                x3.raw_out = phi_out;
                launch_x3<double>(g, x3, ctx->stream);
            }
        }
        ctx->step_rho = nullptr;
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return DFT_OK;
    });
}

dft_status dft_picard_step(dft_ctx *ctx, double *rho_inout, double *alpha_out, double *norm_out) {
    if (!ctx || !rho_inout) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    return guarded([&]() -> dft_status {
        const long long SN = (long long)ctx->geo.S * ctx->geo.N;
        if (ctx->step_rho != rho_inout) {
            DevState h = fresh_state(ctx, 0.0, 1LL << 60);
            write_state(ctx, h);
            launch_copy(ctx->rho0, rho_inout, SN, ctx->stream);
            enqueue_prime(ctx, ctx->stream);
            if (ctx->mixed) ctx->refreshes += 1;
            ctx->step_rho = rho_inout;
        }
        DevState h0 = read_state(ctx);
        if (h0.status) return status_from(h0);
        // a single step always runs (tol = 0 keeps it from reporting convergence early)
        h0.gate_run = 1;
        h0.converged = 0;
        write_state(ctx, h0);
        enqueue_step(ctx, ctx->stream);
        DevState h = read_state(ctx);
        launch_copy(rho_inout, ctx->roles.rho[h.sel & 3], SN, ctx->stream);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (alpha_out) *alpha_out = h.alpha_acc;
        if (norm_out) *norm_out = h.r;
        return status_from(h);
    });
}

dft_status dft_solve(dft_ctx *ctx, double *rho_inout, double tol, int32_t max_iter, int32_t *iters_out,
                     double *norm_out) {
    if (!ctx || !rho_inout) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    if (!(tol >= 0.0) || max_iter < 0) return fail(DFT_E_INVALID_ARG, "tol must be >= 0 and max_iter >= 0");
    return guarded([&]() -> dft_status {
        const long long SN = (long long)ctx->geo.S * ctx->geo.N;
        DevState h = fresh_state(ctx, tol, max_iter);
        write_state(ctx, h);
        launch_copy(ctx->rho0, rho_inout, SN, ctx->stream);
        enqueue_prime(ctx, ctx->stream);
        if (ctx->mixed) ctx->refreshes += 1;
        ensure_graph(ctx);
        const int K = ctx->geo.N >= (1LL << 22) ? 4 : 16;
        h = read_state(ctx);
        double r_ref = h.r;
        double r_prev = h.r;
        bool fp64_checked = true;   // the state's residual comes from an FP64 evaluation
        dft_status out = DFT_OK;
        for (;;) {
            if (h.status) { out = status_from(h); break; }
            if (h.converged) {
                if (fp64_checked) break;
                // FP32-mixed: confirm at the converged iterate with an FP64 evaluation, which
                // also makes it the new reference state
                enqueue_prime(ctx, ctx->stream);
                ctx->refreshes += 1;
                h = read_state(ctx);
                r_ref = h.r;
                fp64_checked = true;
                continue;
            }
            if (h.iters >= max_iter || h.rejected >= 4 * (long long)max_iter + 16) {
                out = fail(DFT_E_NOT_CONVERGED, "max_iter reached");
                break;
            }
            for (int k = 0; k < K; ++k) HIPCHK(hipGraphLaunch(ctx->gexec, ctx->stream));
            h = read_state(ctx);
            fp64_checked = !ctx->mixed;
            if (ctx->mixed && !h.converged && !h.status && (h.r < 1e-4 * r_ref || !(h.r < 0.99 * r_prev))) {
                // refresh the FP64 reference once the residual has fallen far below the
                // reference's, or stalls at the FP32 noise floor
                enqueue_prime(ctx, ctx->stream);
                ctx->refreshes += 1;
                h = read_state(ctx);
                r_ref = h.r;
                fp64_checked = true;
            }
            r_prev = h.r;
        }
        launch_copy(rho_inout, ctx->roles.rho[h.sel & 3], SN, ctx->stream);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->step_rho = rho_inout;
        if (iters_out) *iters_out = (int32_t)h.iters;
        if (norm_out) *norm_out = h.r;
        return out;
    });
}

dft_status dft_run(dft_ctx *ctx, double *rho_inout, int32_t nsteps, int32_t *iters_out, double *norm_out) {
    if (!ctx || !rho_inout) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    if (nsteps < 0) return fail(DFT_E_INVALID_ARG, "nsteps must be >= 0");
    return guarded([&]() -> dft_status {
        const long long SN = (long long)ctx->geo.S * ctx->geo.N;
        if (ctx->step_rho != rho_inout) {
            DevState h = fresh_state(ctx, 0.0, 1LL << 60);
            write_state(ctx, h);
            launch_copy(ctx->rho0, rho_inout, SN, ctx->stream);
            enqueue_prime(ctx, ctx->stream);
            if (ctx->mixed) ctx->refreshes += 1;
            ctx->step_rho = rho_inout;
        }
        DevState h0 = read_state(ctx);
        if (h0.status) return status_from(h0);
        const long long it0 = h0.iters;
        h0.tol = 0.0;
        h0.max_iter = 1LL << 60;
        h0.gate_run = 1;
        h0.converged = 0;
        write_state(ctx, h0);
        ensure_graph(ctx);
        for (int k = 0; k < nsteps; ++k) HIPCHK(hipGraphLaunch(ctx->gexec, ctx->stream));
        DevState h = read_state(ctx);
        launch_copy(rho_inout, ctx->roles.rho[h.sel & 3], SN, ctx->stream);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (iters_out) *iters_out = (int32_t)(h.iters - it0);
        if (norm_out) *norm_out = h.r;
        return status_from(h);
    });
}

dft_status dft_profile(dft_ctx *ctx, const double *rho, int32_t reps, double *ms_out) {
    if (!ctx || !rho || !ms_out || reps < 1) return fail(DFT_E_INVALID_ARG, "bad argument to dft_profile");
    return guarded([&]() -> dft_status {
        if (ctx->mixed && ctx->refreshes == 0) {
            dft_status s2 = dft_set_reference(ctx, rho);
            if (s2 != DFT_OK) return s2;
        }
        hipEvent_t ev[DFT_NPASS + 1];
        for (auto &e : ev) HIPCHK(hipEventCreate(&e));
        std::vector<double> acc(DFT_NPASS, 0.0);
        try {
            for (int r = 0; r < reps; ++r) {
                Eval e;
                e.src = rho;
                e.g_out = ctx->gs;
                e.fslot = &ctx->st->best_f;
                e.fp64 = !ctx->mixed;
                e.count_kind = 0;
                e.events = ev;
                enqueue_eval(ctx, e, ctx->stream);
                HIPCHK(hipEventSynchronize(ev[DFT_NPASS]));
                for (int k = 0; k < DFT_NPASS; ++k) {
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
                    acc[k] += ms;
                }
            }
        } catch (...) {
            for (auto &e : ev) (void)hipEventDestroy(e);
            throw;
        }
        for (auto &e : ev) HIPCHK(hipEventDestroy(e));
        for (int k = 0; k < DFT_NPASS; ++k) ms_out[k] = acc[k] / reps;
        ctx->step_rho = nullptr;
        return DFT_OK;
    });
}

// ------------------------------------------------------------------ implicit adjoint
}  // extern "C"

namespace {

struct AdjLayout {
    size_t nstar, dphi, G, w, r, p, q, Hp, t, wh, rh, dh, th, part, scal, ac, total;
    int nparts;
};

AdjLayout adj_layout(const dft_params *p) {
    AdjLayout L;
    const long long N = (long long)p->n[0] * p->n[1] * p->n[2];
    const long long NC = (long long)(p->n[0] / 2 + 1) * p->n[1] * p->n[2];
    const int S = p->nspecies;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align_up(off + b); return o; };
    const size_t RF = sizeof(double) * (size_t)N, CF = 2 * sizeof(double) * (size_t)NC;
    L.nstar = take(DFT_NALPHA * RF);
    L.dphi = take(DFT_NALPHA * RF);
    L.G = take(S * RF);
    L.w = take(S * RF);
    L.r = take(S * RF);
    L.p = take(S * RF);
    L.q = take(S * RF);
    L.Hp = take(S * RF);
    L.t = take(DFT_NALPHA * RF);
    L.wh = take(S * CF);
    L.rh = take(S * CF);
    L.dh = take(DFT_NALPHA * CF);
    L.th = take(DFT_NALPHA * CF);
    L.nparts = 2048 * DFT_MAX_SPECIES;
    L.part = take(sizeof(double) * (size_t)L.nparts * kAdjNV);
    L.scal = take(sizeof(double) * 64);
    L.ac = take(sizeof(AdjConsts));
    L.total = off;
    return L;
}

// H u = dE/drho . u at the expansion point whose weighted densities are nstar: the residual
// passes in FP64 with the Hessian-vector FMT kernel and no bath subtraction.
void enqueue_hess(dft_ctx *c, const double *u, double *hu, const double *nstar, double *t_out, hipStream_t s) {
    const Geo &g = c->geo;
    XFwdArgs xa{};
    xa.src = u;
    xa.spec = c->specA;
    xa.nfield = g.S;
    xa.mode = XF_PLAIN;
    launch_x_forward<double>(g, xa, s);
    YArgs ya{c->specA, g.S, -1, nullptr};
    launch_y<double>(g, ya, s);
    Z1Args z1{c->specA, c->specB, 0, 1, nullptr};
    launch_z1<double>(g, z1, s);
    YArgs yb{c->specB, DFT_NALPHA, 1, nullptr};
    yb.vec = g.compact ? 1 : 0;
    launch_y<double>(g, yb, s);
    X2Args x2{};
    x2.specB = c->specB;
    x2.hs = c->p.hs_functional;
    x2.mode = X2_HESS;
    x2.nstar = nstar;
    x2.t_out = t_out;
    x2.red = c->red;
    launch_x2<double>(g, x2, s);
    YArgs yc{c->specB, DFT_NALPHA, -1, nullptr};
    yc.vec = g.compact ? 2 : 0;
    launch_y<double>(g, yc, s);
    Z2Args z2{};
    z2.specB = c->specB;
    z2.specA = c->specA;
    z2.mode = Z2_EL;
    launch_z2<double>(g, z2, s);
    YArgs yd{c->specA, g.S, 1, nullptr};
    launch_y<double>(g, yd, s);
    X3Args x3{};
    x3.specA = c->specA;
    x3.nfield = g.S;
    x3.raw = 1;
    x3.raw_out = hu;
    launch_x3<double>(g, x3, s);
}

// Forward 3-D transform (FP64) of nfield contiguous real fields into half spectra.
void forward3d(dft_ctx *c, const double *src, int nfield, void *dst, hipStream_t s) {
    const Geo &g = c->geo;
    XFwdArgs xa{};
    xa.src = src;
    xa.spec = dst;
    xa.nfield = nfield;
    xa.mode = XF_PLAIN;
    launch_x_forward<double>(g, xa, s);
    YArgs ya{dst, nfield, -1, nullptr};
    launch_y<double>(g, ya, s);
    YArgs za{dst, nfield, -1, nullptr, 2};
    launch_y<double>(g, za, s);
}

// Host copy of n <= kMaxScalars device scalars, in a fixed array (no heap allocation).
constexpr int kMaxScalars = 64;
static_assert(kAdjNV <= kMaxScalars, "adjoint reductions exceed the scalar buffer");
struct Scalars {
    double v[kMaxScalars];
    double operator[](int i) const { return v[i]; }
};
Scalars read_scalars(dft_ctx *c, const double *dev, int n) {
    Scalars h;
    HIPCHK(hipMemcpyAsync(h.v, dev, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return h;
}

dft_status adjoint_run(dft_ctx *ctx, const double *rho_star, const double *dO_drho, char *w8, double tol,
                       int32_t max_iter, double *dO_dvext, double *dO_drho_bulk, double *dO_dsigma,
                       int32_t *iters_out, double *resid_out);

}  // namespace

extern "C" {

dft_status dft_adjoint_workspace_size(const dft_params *params, size_t *bytes) {
    std::string msg;
    dft_status st = validate(params, &msg);
    if (st != DFT_OK) return fail(st, msg);
    if (!bytes) return fail(DFT_E_INVALID_ARG, "bytes is NULL");
    *bytes = adj_layout(params).total;
    return DFT_OK;
}

dft_status dft_adjoint(dft_ctx *ctx, const double *rho_star, const double *dO_drho, void *adj_ws, size_t adj_ws_bytes,
                       double tol, int32_t max_iter, double *dO_dvext, double *dO_drho_bulk, double *dO_dsigma,
                       int32_t *iters_out, double *resid_out) {
    if (!ctx || !rho_star || !dO_drho) return fail(DFT_E_INVALID_ARG, "ctx, rho_star or dO_drho is NULL");
    const AdjLayout L = adj_layout(&ctx->p);
    if (!adj_ws || adj_ws_bytes < L.total || ((uintptr_t)adj_ws) % 256 != 0)
        return fail(DFT_E_WORKSPACE, "adjoint workspace missing, misaligned or smaller than dft_adjoint_workspace_size");
    return adjoint_run(ctx, rho_star, dO_drho, (char *)adj_ws, tol, max_iter, dO_dvext, dO_drho_bulk, dO_dsigma,
                       iters_out, resid_out);
}

}  // extern "C"

namespace {

// The implicit adjoint of dft_adjoint with its workspace at w8 (adj_layout bytes, 256-byte aligned).
dft_status adjoint_run(dft_ctx *ctx, const double *rho_star, const double *dO_drho, char *w8, double tol,
                       int32_t max_iter, double *dO_dvext, double *dO_drho_bulk, double *dO_dsigma,
                       int32_t *iters_out, double *resid_out) {
    if (!(tol > 0.0) || max_iter < 1) return fail(DFT_E_INVALID_ARG, "tol must be > 0 and max_iter >= 1");
    const AdjLayout L = adj_layout(&ctx->p);
    if (ctx->geo.S > 4) return fail(DFT_E_UNSUPPORTED_SIZE, "adjoint gradients support at most 4 species");
    if ((size_t)DFT_NALPHA * ctx->geo.nx * 16 > 65536)
        return fail(DFT_E_UNSUPPORTED_SIZE, "adjoint needs n_x <= 384 (FP64 Hessian pass)");
    return guarded([&]() -> dft_status {
        dft_ctx *c = ctx;
        const Geo &g = c->geo;
        const int S = g.S;
        const long long N = g.N, SN = (long long)S * N;
        hipStream_t s = c->stream;
        double *nstar = (double *)(w8 + L.nstar), *dphi = (double *)(w8 + L.dphi), *G = (double *)(w8 + L.G);
        double *w = (double *)(w8 + L.w), *r = (double *)(w8 + L.r), *p = (double *)(w8 + L.p);
        double *q = (double *)(w8 + L.q), *Hp = (double *)(w8 + L.Hp), *t = (double *)(w8 + L.t);
        double *part = (double *)(w8 + L.part), *scal = (double *)(w8 + L.scal);
        AdjConsts *acd = (AdjConsts *)(w8 + L.ac);
        // FP64 evaluation at rho*: G*, n*, dPhi(n*)
        Eval e;
        e.src = rho_star;
        e.g_out = G;
        e.n_out = nstar;
        e.dphi_out = dphi;
        e.fslot = &c->st->best_f;
        e.fp64 = true;
        e.count_kind = 0;
        enqueue_eval(c, e, s);
        // ||g|| on fluid nodes via the (r, r) partial of r0 with Hw := g
        int nb = adj_r0(SN, G, dO_drho, r, p, part, s);
        adj_reduce(part, nb, 2, scal, s);
        const double gnorm = std::sqrt(read_scalars(c, scal, 2)[1]);
        if (!(gnorm > 0.0)) return fail(DFT_E_INVALID_ARG, "dO_drho vanishes on every fluid node");
        // w0 = G o g, r0 = g - (w0/G - H w0) = H w0, p0 = G o r0
        adj_init(SN, G, dO_drho, w, s);
        enqueue_hess(c, w, Hp, nstar, nullptr, s);
        nb = adj_r0(SN, G, Hp, r, p, part, s);
        adj_reduce(part, nb, 2, scal, s);
        Scalars sc = read_scalars(c, scal, 2);
        double rz = sc[0], rr = sc[1];
        int it = 0;
        double rel = std::sqrt(rr) / gnorm;
        while (rel > tol && it < max_iter) {
            enqueue_hess(c, p, Hp, nstar, nullptr, s);
            nb = adj_q(SN, G, p, Hp, q, part, s);
            adj_reduce(part, nb, 1, scal, s);
            const double pq = read_scalars(c, scal, 1)[0];
            if (!(pq > 0.0)) return fail(DFT_E_NONFINITE, "adjoint system is not positive definite at rho*");
            const double alpha = rz / pq;
            nb = adj_step(SN, alpha, G, p, q, w, r, part, s);
            adj_reduce(part, nb, 2, scal, s);
            sc = read_scalars(c, scal, 2);
            const double rz_new = sc[0];
            rr = sc[1];
            adj_dir(SN, rz_new / rz, G, r, p, s);
            rz = rz_new;
            rel = std::sqrt(rr) / gnorm;
            ++it;
            if (!std::isfinite(rel)) return fail(DFT_E_NONFINITE, "non-finite adjoint residual");
        }
        if (iters_out) *iters_out = it;
        if (resid_out) *resid_out = rel;
        if (rel > tol) return fail(DFT_E_NOT_CONVERGED, "adjoint solve reached max_iter");
        if (dO_dvext) adj_neg(SN, w, dO_dvext, s);
        if (!dO_drho_bulk && !dO_dsigma) {
            HIPCHK(hipStreamSynchronize(s));
            return DFT_OK;
        }
        // t = Phi''(n*) (A w) for the final w
        enqueue_hess(c, w, Hp, nstar, t, s);
        // W_i = sum_x w_i
        nb = adj_fieldsum(N, S, w, part, s);
        double Wsum[DFT_MAX_SPECIES] = {};
        for (int i = 0; i < S; ++i) {
            adj_reduce(part + (long long)i * nb, nb, 1, scal + i, s);
        }
        sc = read_scalars(c, scal, S);
        for (int i = 0; i < S; ++i) Wsum[i] = sc[i];
        // spectra of w, rho*, dPhi(n*) and t
        forward3d(c, w, S, w8 + L.wh, s);
        forward3d(c, rho_star, S, w8 + L.rh, s);
        forward3d(c, dphi, DFT_NALPHA, w8 + L.dh, s);
        forward3d(c, t, DFT_NALPHA, w8 + L.th, s);
        // kernel-coefficient derivatives with respect to lambda_i, lambda_j
        const dft_bulk_info &b = c->bulk;
        AdjConsts ac;
        std::memset(&ac, 0, sizeof ac);
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) {
                const int ij = i * DFT_MAX_SPECIES + j;
                if (!c->p.electrostatics) continue;
                const double li = b.lambda[i], lj = b.lambda[j];
                const double pre = 0.5 * c->p.valence[i] * c->p.valence[j] * c->p.bjerrum_length;
                ac.li_c1[ij] = -pre / (2.0 * li * li * lj);
                ac.lj_c1[ij] = -pre / (2.0 * li * lj * lj);
                ac.li_c0[ij] = pre / (li * li);
                ac.lj_c0[ij] = pre / (lj * lj);
                ac.li_cm1[ij] = 0.5 * pre * (1.0 / lj - lj / (li * li));
                ac.lj_cm1[ij] = 0.5 * pre * (1.0 / li - li / (lj * lj));
            }
        HIPCHK(hipMemcpyAsync(acd, &ac, sizeof ac, hipMemcpyHostToDevice, s));
        AdjSpecArgs sa{w8 + L.wh, w8 + L.rh, w8 + L.dh, w8 + L.th, acd, part};
        nb = adj_spec(g, sa, s);
        adj_reduce(part, nb, kAdjNV, scal, s);
        sc = read_scalars(c, scal, kAdjNV);
        const double invN = 1.0 / (double)N;
        BulkDeriv bd;
        bulk_derivatives(&c->p, b, &bd);
        auto B = [&](int i, int j, int m) { return sc[4 + 3 * (i * 4 + j) + m] * invN; };
        double Bgam = 0.0;   // sum_ij <w_i, dC_ij/dGamma * drho_j>
        if (c->p.electrostatics) {
            const double G2 = b.gamma * b.gamma;
            const double dRc = (c->p.flags & DFT_FLAG_CUTOFF_LAMBDA) ? -1.0 / G2 : 0.0;
            for (int i = 0; i < S; ++i)
                for (int j = 0; j < S; ++j) Bgam += -(B(i, j, 0) + B(i, j, 1)) / (2.0 * G2) + B(i, j, 2) * dRc;
        }
        for (int k = 0; k < S; ++k) {
            double dr = Wsum[k] / c->p.rho_bulk[k];
            double dR = 0.0;
            for (int i = 0; i < S; ++i) {
                dr += Wsum[i] * bd.dmu_drho[i][k];
                dR += Wsum[i] * 2.0 * bd.dmu_dsigma[i][k];
            }
            dR -= sc[k] * invN;
            if (c->p.electrostatics) {
                for (int i = 0; i < S; ++i) {
                    const int ik = i * DFT_MAX_SPECIES + k;
                    const double Rc = c->hc.sc_R[ik];
                    const double C0 = c->hc.sc_c1[ik] * M_PI * Rc * Rc * Rc * Rc +
                                      c->hc.sc_c0[ik] * 4.0 * M_PI * Rc * Rc * Rc / 3.0 +
                                      c->hc.sc_cm1[ik] * 2.0 * M_PI * Rc * Rc;
                    dr -= Wsum[i] * C0;
                }
                dr += bd.dgamma_drho[k] * Bgam;
                for (int j = 0; j < S; ++j) dR += B(k, j, 0) + B(k, j, 2);
                for (int i = 0; i < S; ++i) dR += B(i, k, 1) + B(i, k, 2);
                dR += 2.0 * bd.dgamma_dsigma[k] * Bgam;
            }
            if (dO_drho_bulk) dO_drho_bulk[k] = dr;
            if (dO_dsigma) dO_dsigma[k] = 0.5 * dR;
        }
        return DFT_OK;
    });
}

// ------------------------------------------------------------------ adjoint without allocation
// dft_adjoint_noalloc keeps its workspace in this array of the library's device image, one copy
// per GPU, resident until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns on each device (kept in scratch_dev); the array's name is a host
// stand-in, never a device address.
__device__ __align__(256) char scratch[DFT_ADJOINT_NOALLOC_MAX_BYTES];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *scratch_dev[kScratchDevices] = {};

// The current device's copy of the scratch array, looked up on the device's first call.
dft_status scratch_address(char **out) {
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DFT_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kScratchDevices) return fail(DFT_E_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e2 = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e2 != hipSuccess || !p)
            return fail(DFT_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e2));
        scratch_dev[dev] = p;
    }
    *out = (char *)scratch_dev[dev];
    return DFT_OK;
}

}  // namespace

extern "C" {

dft_status dft_adjoint_noalloc(dft_ctx *ctx, const double *rho_star, const double *dO_drho, double tol,
                               int32_t max_iter, double *dO_dvext, double *dO_drho_bulk, double *dO_dsigma,
                               int32_t *iters_out, double *resid_out) {
    if (!ctx || !rho_star || !dO_drho) return fail(DFT_E_INVALID_ARG, "ctx, rho_star or dO_drho is NULL");
    const AdjLayout L = adj_layout(&ctx->p);
    if (L.total > (size_t)DFT_ADJOINT_NOALLOC_MAX_BYTES)
        return fail(DFT_E_WORKSPACE, "problem needs more adjoint workspace than DFT_ADJOINT_NOALLOC_MAX_BYTES; "
                                     "use dft_adjoint with a caller workspace");
    char *w8 = nullptr;
    const dft_status st = scratch_address(&w8);
    if (st != DFT_OK) return st;
    return adjoint_run(ctx, rho_star, dO_drho, w8, tol, max_iter, dO_dvext, dO_drho_bulk, dO_dsigma, iters_out,
                       resid_out);
}

// ------------------------------------------------------------------ Newton-Krylov
dft_status dft_newton(dft_ctx *ctx, double *rho, void *adj_ws, size_t adj_ws_bytes, double tol, int32_t max_iter,
                      int32_t *iters_out, int32_t *cg_iters_out, double *norm_out) {
    if (!ctx || !rho) return fail(DFT_E_INVALID_ARG, "ctx or rho is NULL");
    if (!(tol > 0.0) || max_iter < 0) return fail(DFT_E_INVALID_ARG, "tol must be > 0 and max_iter >= 0");
    const AdjLayout L = adj_layout(&ctx->p);
    if (!adj_ws || adj_ws_bytes < L.total || ((uintptr_t)adj_ws) % 256 != 0)
        return fail(DFT_E_WORKSPACE, "Newton workspace missing, misaligned or smaller than dft_adjoint_workspace_size");
    if (ctx->geo.S > 4) return fail(DFT_E_UNSUPPORTED_SIZE, "Newton-Krylov supports at most 4 species");
    if ((size_t)DFT_NALPHA * ctx->geo.nx * 16 > 65536)
        return fail(DFT_E_UNSUPPORTED_SIZE, "Newton-Krylov needs n_x <= 384 (FP64 Hessian pass)");
    return guarded([&]() -> dft_status {
        dft_ctx *c = ctx;
        const Geo &g = c->geo;
        const long long SN = (long long)g.S * g.N;
        hipStream_t s = c->stream;
        char *w8 = (char *)adj_ws;
        double *nstar = (double *)(w8 + L.nstar), *G = (double *)(w8 + L.G), *rhs = (double *)(w8 + L.dphi);
        double *d = (double *)(w8 + L.w), *r = (double *)(w8 + L.r), *p = (double *)(w8 + L.p);
        double *q = (double *)(w8 + L.q), *Hp = (double *)(w8 + L.Hp);
        double *part = (double *)(w8 + L.part), *scal = (double *)(w8 + L.scal);
        double *trial = c->rho_t;
        const double nfl = c->hc.nfluid, cap = c->hc.eta_cap;
        c->step_rho = nullptr;   // the Picard state no longer describes the caller's density
        // FP64 evaluation: G and n at src, f and max n3 into the state's scratch slots
        auto evaluate = [&](const double *src, double &f, double &m) {
            Eval e;
            e.src = src;
            e.g_out = G;
            e.n_out = nstar;
            e.fslot = &c->st->fb;
            e.mslot = &c->st->mb;
            e.fp64 = true;
            e.count_kind = 0;
            enqueue_eval(c, e, s);
            const Scalars fm = read_scalars(c, &c->st->fb, 2);
            f = fm[0];
            m = fm[1];
        };
        double f, m;
        evaluate(rho, f, m);
        double res = std::sqrt(f / nfl), res_prev = res;
        int it = 0, cg_total = 0;
        while (it < max_iter && res > tol) {
            if (!std::isfinite(f)) return fail(DFT_E_NONFINITE, "non-finite residual at the current iterate");
            if (!(m < cap)) return fail(DFT_E_PACKING, "max n3 reached the packing cap at the current iterate");
            // (diag(G)^-1 - H) d = (G - rho) / G by CG preconditioned with diag(G), from the
            // Picard direction d0 = G - rho; forcing term shrinks with the residual
            newton_rhs(SN, G, rho, rhs, s);
            int nb = adj_r0(SN, G, rhs, r, p, part, s);
            adj_reduce(part, nb, 2, scal, s);
            const double gnorm = std::sqrt(read_scalars(c, scal, 2)[1]);
            adj_init(SN, G, rhs, d, s);
            const double eta = std::max(1e-10, std::min(0.1, it == 0 ? 0.1 : 0.9 * (res / res_prev) * (res / res_prev)));
            if (gnorm > 0.0) {
                enqueue_hess(c, d, Hp, nstar, nullptr, s);
                nb = adj_r0(SN, G, Hp, r, p, part, s);
                adj_reduce(part, nb, 2, scal, s);
                Scalars sc = read_scalars(c, scal, 2);
                double rz = sc[0], rel = std::sqrt(sc[1]) / gnorm;
                for (int k = 0; k < 500 && rel > eta; ++k) {
                    enqueue_hess(c, p, Hp, nstar, nullptr, s);
                    nb = adj_q(SN, G, p, Hp, q, part, s);
                    adj_reduce(part, nb, 1, scal, s);
                    const double pq = read_scalars(c, scal, 1)[0];
                    if (!(pq > 0.0)) break;   // not positive definite here: keep the current direction
                    const double alpha = rz / pq;
                    nb = adj_step(SN, alpha, G, p, q, d, r, part, s);
                    adj_reduce(part, nb, 2, scal, s);
                    sc = read_scalars(c, scal, 2);
                    adj_dir(SN, sc[0] / rz, G, r, p, s);
                    rz = sc[0];
                    rel = std::sqrt(sc[1]) / gnorm;
                    ++cg_total;
                    if (!std::isfinite(rel)) return fail(DFT_E_NONFINITE, "non-finite Newton-Krylov residual");
                }
            }
            // largest step keeping every density positive, then backtracking on f
            nb = newton_bound(SN, rho, d, part, s);
            std::vector<double> mins(nb);
            HIPCHK(hipMemcpyAsync(mins.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            double lam_pos = INFINITY;
            for (double v : mins) lam_pos = std::min(lam_pos, v);
            double lam = std::min(1.0, 0.9 * lam_pos);
            bool accepted = false;
            for (int ls = 0; ls < 40 && lam > 0.0; ++ls) {
                axpy(SN, rho, lam, d, trial, s);
                double ft, mt;
                evaluate(trial, ft, mt);
                if (mt < cap && std::isfinite(ft) && ft <= (1.0 - 1e-4 * lam) * f) {
                    launch_copy(rho, trial, SN, s);
                    f = ft;
                    m = mt;
                    accepted = true;
                    break;
                }
                lam *= 0.5;
            }
            if (!accepted) {
                evaluate(rho, f, m);   // G and n of the caller's density again
                return fail(DFT_E_NOT_CONVERGED, "Newton line search found no decrease of the residual");
            }
            res_prev = res;
            res = std::sqrt(f / nfl);
            ++it;
        }
        HIPCHK(hipStreamSynchronize(s));
        if (iters_out) *iters_out = it;
        if (cg_iters_out) *cg_iters_out = cg_total;
        if (norm_out) *norm_out = res;
        if (res > tol) return fail(DFT_E_NOT_CONVERGED, "Newton-Krylov reached max_iter");
        return DFT_OK;
    });
}

dft_status dft_rfd_reference(dft_ctx *ctx, const double *f, const double *rsc, int32_t nodes, double *f_ref) {
    if (!ctx || !f || !rsc || !f_ref) return fail(DFT_E_INVALID_ARG, "ctx, f, rsc or f_ref is NULL");
    if (nodes < 1 || nodes > DFT_RFD_MAX_NODES) return fail(DFT_E_INVALID_ARG, "nodes must lie in 1 .. DFT_RFD_MAX_NODES");
    if (ctx->geo.nprob != 1) return fail(DFT_E_INVALID_ARG, "a batch group ctx holds several points; use a member ctx");
    return guarded([&]() -> dft_status {
        dft_ctx *c = ctx;
        const Geo &g = c->geo;
        hipStream_t s = c->stream;
        // range of R_SC (and its validity) on the host
        const int nb = rsc_range(g.N, rsc, c->red.fpart, c->red.mpart, c->red.fflag, c->red.cap, s);
        std::vector<double> lo(nb), hi(nb);
        std::vector<int> bad(nb);
        HIPCHK(hipMemcpyAsync(lo.data(), c->red.fpart, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hi.data(), c->red.mpart, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(bad.data(), c->red.fflag, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double rlo = INFINITY, rhi = -INFINITY;
        long long nbad = 0;
        for (int i = 0; i < nb; ++i) {
            rlo = std::min(rlo, lo[i]);
            rhi = std::max(rhi, hi[i]);
            nbad += bad[i];
        }
        if (nbad) return fail(DFT_E_INVALID_ARG, "rsc must be positive and finite at every node");
        // Chebyshev points of the range (one point when R_SC is constant)
        int M = nodes;
        if (!(rhi - rlo > 1e-15 * rhi)) M = 1;
        const double cc = 0.5 * (rlo + rhi), dd = M == 1 ? 0.0 : 0.5 * (rhi - rlo);
        // forward x, y transforms of the S fields (FP64), kept in specA for every radius
        XFwdArgs xa{};
        xa.src = f;
        xa.spec = c->specA;
        xa.nfield = g.S;
        xa.mode = XF_PLAIN;
        launch_x_forward<double>(g, xa, s);
        YArgs ya{c->specA, g.S, -1, nullptr};
        launch_y<double>(g, ya, s);
        // scratch in the line-search roles that do not hold the current iterate (kept)
        const int sel = read_state(c).sel & 3;
        double *inv_den = c->roles.G[(sel + 1) & 3];
        int *hit = reinterpret_cast<int *>(c->roles.G[(sel + 2) & 3]);
        double *raw = c->roles.rho[(sel + 1) & 3];
        cheb_prep(g.N, rsc, M, cc, dd, inv_den, hit, s);
        for (int m = 0; m < M; ++m) {
            const double Rm = cc + dd * std::cos(M_PI * (2.0 * m + 1.0) / (2.0 * M));
            Z2Args z2{};
            z2.specA = c->specA;
            z2.specB = c->specB;
            z2.mode = Z2_BALL;
            z2.nsrc = g.S;
            z2.radius = Rm;
            launch_z2<double>(g, z2, s);
            YArgs yb{c->specB, g.S, 1, nullptr};
            launch_y<double>(g, yb, s);
            X3Args x3{};
            x3.specA = c->specB;
            x3.nfield = g.S;
            x3.raw = 1;
            x3.raw_out = raw;
            launch_x3<double>(g, x3, s);
            cheb_accum(g.N, g.S, m, M, cc, dd, rsc, inv_den, hit, raw, f_ref, m == 0, s);
        }
        return DFT_OK;
    });
}

// ------------------------------------------------------------------ batches of state points
struct dft_batch {
    std::vector<dft_ctx *> members;   // caller order; each owns a slice of the batch workspace
    struct Group {
        std::vector<int> idx;         // members sharing launch choices (see same_shape)
        dft_ctx *lead = nullptr;      // geometry covering the whole group (nprob, pstride)
        long long stride = 0;
        int rec = 0;                  // the group's first record in the state mirror
        hipStream_t stream = nullptr; // the group's work stream (one of gstreams)
    };
    std::vector<Group> groups;
    hipStream_t stream = nullptr;     // the caller's stream
    // Groups run concurrently on up to kBatchStreams streams of default priority, ordered after
    // the caller's stream at the start of a solve and before it at the end.
    std::vector<hipStream_t> gstreams;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    // Line-search states of all members, group by group: gathered on the device into one array
    // and read by the host with one copy per group (pinned host mirror); refresh gates the same way.
    DevState *mirror_dev = nullptr;
    int *gates_dev = nullptr;
    DevState *mirror_host = nullptr;
    int *gates_host = nullptr;
};

namespace {

// Points of one group share the launch choices of its lead: grid, species count, precision,
// functional, electrostatics on/off and the screening cutoff.
bool same_shape(const dft_params &a, const dft_params &b) {
    return a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2] && a.nspecies == b.nspecies &&
           a.precision == b.precision && a.hs_functional == b.hs_functional &&
           a.electrostatics == b.electrostatics &&
           (a.flags & DFT_FLAG_CUTOFF_LAMBDA) == (b.flags & DFT_FLAG_CUTOFF_LAMBDA);
}

constexpr int kBatchStreams = 4;

// Groups (first-seen order), the byte offset of every member in the batch workspace, and the
// offsets of the state mirror (count records) and refresh gates (count ints) after them.
size_t batch_plan(const dft_params *params, int count, std::vector<dft_batch::Group> *groups,
                  std::vector<size_t> *offsets, size_t *mirror_off = nullptr, size_t *gates_off = nullptr) {
    groups->clear();
    offsets->assign(count, 0);
    for (int i = 0; i < count; ++i) {
        bool placed = false;
        for (auto &g : *groups)
            if (same_shape(params[g.idx[0]], params[i])) { g.idx.push_back(i); placed = true; break; }
        if (!placed) {
            dft_batch::Group g;
            g.idx.push_back(i);
            groups->push_back(g);
        }
    }
    size_t off = 0;
    int rec = 0;
    for (auto &g : *groups) {
        g.stride = (long long)make_layout(&params[g.idx[0]]).total;
        g.rec = rec;
        rec += (int)g.idx.size();
        for (size_t m = 0; m < g.idx.size(); ++m) (*offsets)[g.idx[m]] = off + m * (size_t)g.stride;
        off += g.idx.size() * (size_t)g.stride;
    }
    if (mirror_off) *mirror_off = off;
    off = align_up(off + sizeof(DevState) * (size_t)count);
    if (gates_off) *gates_off = off;
    off = align_up(off + sizeof(int) * (size_t)count);
    return off;
}

}  // namespace

dft_status dft_batch_workspace_size(const dft_params *params, int32_t count, size_t *bytes) {
    if (!params || count < 1 || !bytes) return fail(DFT_E_INVALID_ARG, "params, count or bytes invalid");
    std::string msg;
    for (int i = 0; i < count; ++i) {
        dft_status st = validate(&params[i], &msg);
        if (st != DFT_OK) return fail(st, "state point " + std::to_string(i) + ": " + msg);
    }
    std::vector<dft_batch::Group> groups;
    std::vector<size_t> offs;
    *bytes = batch_plan(params, count, &groups, &offs);
    return DFT_OK;
}

dft_status dft_setup_batch(const dft_params *params, int32_t count, const double *const *beta_vext,
                           const double *const *fixed_charge, void *workspace, size_t ws_bytes, void *stream,
                           dft_batch **out) {
    if (!out) return fail(DFT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    dft_status st = dft_batch_workspace_size(params, count, &need);
    if (st != DFT_OK) return st;
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace) % 256 != 0)
        return fail(DFT_E_WORKSPACE, "batch workspace missing, misaligned or smaller than dft_batch_workspace_size");
    dft_batch *b = new dft_batch();
    b->stream = (hipStream_t)stream;
    std::vector<size_t> offs;
    size_t moff = 0, goff = 0;
    batch_plan(params, count, &b->groups, &offs, &moff, &goff);
    b->mirror_dev = (DevState *)((char *)workspace + moff);
    b->gates_dev = (int *)((char *)workspace + goff);
    for (int i = 0; i < count; ++i) {
        dft_ctx *c = nullptr;
        st = dft_setup(&params[i], beta_vext ? beta_vext[i] : nullptr, fixed_charge ? fixed_charge[i] : nullptr,
                       (char *)workspace + offs[i], ws_bytes - offs[i], stream, &c);
        if (st != DFT_OK) {
            std::string m = dft_last_error();
            dft_batch_destroy(b);
            return fail(st, "state point " + std::to_string(i) + ": " + m);
        }
        b->members.push_back(c);
    }
    for (auto &g : b->groups) {
        dft_ctx *lead = new dft_ctx(*b->members[g.idx[0]]);
        lead->graph = nullptr;
        lead->gexec = nullptr;
        lead->cap_stream = nullptr;
        lead->geo.nprob = (int)g.idx.size();
        lead->geo.pstride = g.stride;
        g.lead = lead;
    }
    // launch shapes for the whole group (the members' spectra are scratch here); group streams,
    // events and the pinned state mirror
    st = guarded([&]() -> dft_status {
        const int ns = std::min<int>((int)b->groups.size(), kBatchStreams);
        for (int k = 0; k < ns; ++k) {
            hipStream_t gs = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
            b->gstreams.push_back(gs);
            hipEvent_t ev = nullptr;
            HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            b->joins.push_back(ev);
        }
        HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (size_t k = 0; k < b->groups.size(); ++k) b->groups[k].stream = b->gstreams[k % ns];
        HIPCHK(hipHostMalloc((void **)&b->mirror_host, sizeof(DevState) * (size_t)count, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&b->gates_host, sizeof(int) * (size_t)count, hipHostMallocDefault));
        for (auto &g : b->groups) {
            dft_ctx *lead = g.lead;
            if (lead->geo.nprob > 1 && !(lead->p.flags & DFT_FLAG_NO_AUTOTUNE))
                autotune(lead->geo, TuneBufs{lead->specA, 0, lead->specB, 0}, true, lead->mixed, lead->stream);
        }
        return DFT_OK;
    });
    if (st != DFT_OK) {
        std::string m = dft_last_error();
        dft_batch_destroy(b);
        return fail(st, m);
    }
    *out = b;
    g_last_error.clear();
    return DFT_OK;
}

dft_status dft_batch_member(dft_batch *batch, int32_t i, dft_ctx **out) {
    if (!batch || !out || i < 0 || i >= (int)batch->members.size()) return fail(DFT_E_INVALID_ARG, "bad batch index");
    *out = batch->members[i];
    return DFT_OK;
}

dft_status dft_solve_batch(dft_batch *batch, double *const *rho_inout, double tol, int32_t max_iter,
                           int32_t *iters_out, double *norm_out, int32_t *status_out) {
    if (!batch || !rho_inout) return fail(DFT_E_INVALID_ARG, "batch or rho is NULL");
    if (!(tol >= 0.0) || max_iter < 0) return fail(DFT_E_INVALID_ARG, "tol must be >= 0 and max_iter >= 0");
    const int n = (int)batch->members.size();
    for (int i = 0; i < n; ++i)
        if (!rho_inout[i]) return fail(DFT_E_INVALID_ARG, "rho_inout has a NULL entry");
    return guarded([&]() -> dft_status {
        hipStream_t s = batch->stream;
        DevState *hm = batch->mirror_host;
        std::vector<int> rec(n);
        for (auto &g : batch->groups)
            for (size_t m = 0; m < g.idx.size(); ++m) rec[g.idx[m]] = g.rec + (int)m;
        std::vector<DevState> h(n);
        std::vector<double> r_ref(n), r_prev(n);
        std::vector<char> checked(n, 1), done(n, 0);
        std::vector<int> stat(n, DFT_OK);
        auto first_state = [&](const dft_batch::Group &g) { return batch->members[g.idx[0]]->st; };
        // every group's states: gathered on its stream, one copy per group, then one wait per stream
        auto read_all = [&]() {
            for (auto &g : batch->groups) {
                const int m = (int)g.idx.size();
                launch_copy_states(batch->mirror_dev + g.rec, (long long)sizeof(DevState), first_state(g), g.stride,
                                   m, g.stream);
                HIPCHK(hipMemcpyAsync(hm + g.rec, batch->mirror_dev + g.rec, sizeof(DevState) * m,
                                      hipMemcpyDeviceToHost, g.stream));
            }
            for (hipStream_t gs : batch->gstreams) HIPCHK(hipStreamSynchronize(gs));
            for (int i = 0; i < n; ++i) h[i] = hm[rec[i]];
        };
        // the group streams start after the caller's earlier work
        HIPCHK(hipEventRecord(batch->fork, s));
        for (hipStream_t gs : batch->gstreams) HIPCHK(hipStreamWaitEvent(gs, batch->fork, 0));
        for (auto &g : batch->groups) {
            const int m = (int)g.idx.size();
            for (int k = 0; k < m; ++k) {
                dft_ctx *c = batch->members[g.idx[k]];
                hm[g.rec + k] = fresh_state(c, tol, max_iter);
                launch_copy(c->rho0, rho_inout[g.idx[k]], (long long)c->geo.S * c->geo.N, g.stream);
                c->step_rho = nullptr;
            }
            HIPCHK(hipMemcpyAsync(batch->mirror_dev + g.rec, hm + g.rec, sizeof(DevState) * m, hipMemcpyHostToDevice,
                                  g.stream));
            launch_copy_states(first_state(g), g.stride, batch->mirror_dev + g.rec, (long long)sizeof(DevState), m,
                               g.stream);
            enqueue_prime(g.lead, g.stream);
            for (int i : g.idx)
                if (batch->members[i]->mixed) batch->members[i]->refreshes += 1;
            ensure_graph(g.lead);
        }
        read_all();
        for (int i = 0; i < n; ++i) r_ref[i] = r_prev[i] = h[i].r;
        for (;;) {
            // classify, and choose the members that need an FP64 (reference) evaluation
            std::vector<char> refresh(n, 0);
            bool any_active = false;
            for (int i = 0; i < n; ++i) {
                if (done[i]) continue;
                const bool mixed = batch->members[i]->mixed;
                if (h[i].status) { stat[i] = h[i].status; done[i] = 1; continue; }
                if (h[i].converged) {
                    if (checked[i]) { done[i] = 1; continue; }
                    refresh[i] = 1;
                } else if (h[i].iters >= max_iter || h[i].rejected >= 4 * (long long)max_iter + 16) {
                    stat[i] = DFT_E_NOT_CONVERGED;
                    done[i] = 1;
                    continue;
                } else if (mixed && !checked[i] && (h[i].r < 1e-4 * r_ref[i] || !(h[i].r < 0.99 * r_prev[i]))) {
                    refresh[i] = 1;
                }
                any_active = true;
            }
            if (!any_active) break;
            bool any_refresh = false;
            for (auto &g : batch->groups) {
                bool gr = false;
                for (int i : g.idx) gr |= refresh[i] != 0;
                if (!gr) continue;
                any_refresh = true;
                const int m = (int)g.idx.size();
                for (int k = 0; k < m; ++k) batch->gates_host[g.rec + k] = refresh[g.idx[k]];
                HIPCHK(hipMemcpyAsync(batch->gates_dev + g.rec, batch->gates_host + g.rec, sizeof(int) * m,
                                      hipMemcpyHostToDevice, g.stream));
                launch_set_gates(first_state(g), g.stride, m, batch->gates_dev + g.rec, g.stream);
                enqueue_prime(g.lead, g.stream, true);
            }
            if (any_refresh) {
                read_all();
                for (int i = 0; i < n; ++i) {
                    if (!refresh[i]) continue;
                    r_ref[i] = h[i].r;
                    checked[i] = 1;
                    batch->members[i]->refreshes += 1;
                }
                continue;
            }
            for (auto &g : batch->groups) {
                bool active = false;
                for (int i : g.idx) active |= !done[i];
                if (!active) continue;
                long long ntot = 0;
                for (int i : g.idx) ntot += batch->members[i]->geo.N;
                const int K = ntot >= (1LL << 22) ? 4 : 16;
                for (int k = 0; k < K; ++k) HIPCHK(hipGraphLaunch(g.lead->gexec, g.stream));
            }
            std::vector<double> r_last(n);
            for (int i = 0; i < n; ++i) r_last[i] = h[i].r;
            read_all();
            for (int i = 0; i < n; ++i) {
                if (done[i]) continue;
                r_prev[i] = r_last[i];
                checked[i] = !batch->members[i]->mixed;
            }
        }
        dft_status out = DFT_OK;
        for (auto &g : batch->groups)
            for (int i : g.idx) {
                dft_ctx *c = batch->members[i];
                launch_copy(rho_inout[i], c->roles.rho[h[i].sel & 3], (long long)c->geo.S * c->geo.N, g.stream);
                c->step_rho = rho_inout[i];
                c->stream = s;
            }
        // the caller's stream continues after every group's work
        for (size_t k = 0; k < batch->gstreams.size(); ++k) {
            HIPCHK(hipEventRecord(batch->joins[k], batch->gstreams[k]));
            HIPCHK(hipStreamWaitEvent(s, batch->joins[k], 0));
        }
        for (int i = 0; i < n; ++i) {
            if (iters_out) iters_out[i] = (int32_t)h[i].iters;
            if (norm_out) norm_out[i] = h[i].r;
            if (status_out) status_out[i] = stat[i];
            if (stat[i] != DFT_OK && out == DFT_OK) out = (dft_status)stat[i];
        }
        HIPCHK(hipStreamSynchronize(s));
        if (out != DFT_OK) return fail(out, "at least one state point did not converge (see status_out)");
        return DFT_OK;
    });
}

dft_status dft_batch_destroy(dft_batch *batch) {
    if (!batch) return DFT_OK;
    for (hipStream_t gs : batch->gstreams) (void)hipStreamDestroy(gs);
    for (hipEvent_t ev : batch->joins) (void)hipEventDestroy(ev);
    if (batch->fork) (void)hipEventDestroy(batch->fork);
    if (batch->mirror_host) (void)hipHostFree(batch->mirror_host);
    if (batch->gates_host) (void)hipHostFree(batch->gates_host);
    for (auto &g : batch->groups) {
        if (!g.lead) continue;
        if (g.lead->gexec) (void)hipGraphExecDestroy(g.lead->gexec);
        if (g.lead->graph) (void)hipGraphDestroy(g.lead->graph);
        if (g.lead->cap_stream) (void)hipStreamDestroy(g.lead->cap_stream);
        delete g.lead;
    }
    for (dft_ctx *c : batch->members) dft_destroy(c);
    delete batch;
    return DFT_OK;
}

dft_status dft_get_stats(dft_ctx *ctx, dft_stats *out) {
    if (!ctx || !out) return fail(DFT_E_INVALID_ARG, "ctx or out is NULL");
    return guarded([&]() -> dft_status {
        DevState h = read_state(ctx);
        out->iterations = h.iters;
        out->rejected = h.rejected;
        out->g_evals = h.gevals;
        out->n3_evals = h.n3evals;
        out->fp64_refresh = ctx->refreshes;
        out->residual = h.r;
        out->alpha = h.alpha_acc;
        out->max_n3 = h.m0;
        out->step_cap = h.cap;
        out->compact_layout = ctx->geo.compact;
        return DFT_OK;
    });
}

dft_status dft_get_schedule(const dft_ctx *ctx, int32_t *shapes_out) {
    if (!ctx || !shapes_out) return fail(DFT_E_INVALID_ARG, "ctx or shapes_out is NULL");
    for (int p = 0; p < DFT_TUNE_PASSES; ++p)
        for (int t = 0; t < 2; ++t) shapes_out[2 * p + t] = ctx->geo.tune[p][t];
    return DFT_OK;
}

dft_status dft_set_schedule(dft_ctx *ctx, const int32_t *shapes) {
    if (!ctx || !shapes) return fail(DFT_E_INVALID_ARG, "ctx or shapes is NULL");
    const Geo &g = ctx->geo;
    const int ny_v = g.ny > 1 ? y_ct_variants(g.ny, false) : 0;
    const int nv[DFT_TUNE_PASSES] = {ny_v, g.nz > 1 ? y_ct_variants(g.nz, false) : 0, z1_ct_variants(g.nz),
                                     z_ct_variants(g.nz), ny_v, ny_v};
    for (int p = 0; p < DFT_TUNE_PASSES; ++p)
        for (int t = 0; t < 2; ++t) {
            const int v = shapes[2 * p + t];
            if (v < 0 || v >= std::max(nv[p], 1)) {
                char buf[120];
                snprintf(buf, sizeof buf, "shape %d of pass %d outside 0..%d", v, p, std::max(nv[p], 1) - 1);
                return fail(DFT_E_INVALID_ARG, buf);
            }
        }
    return guarded([&]() -> dft_status {
        for (int p = 0; p < DFT_TUNE_PASSES; ++p)
            for (int t = 0; t < 2; ++t) ctx->geo.tune[p][t] = shapes[2 * p + t];
        // the captured step graph holds the old launches
        if (ctx->gexec) HIPCHK(hipGraphExecDestroy(ctx->gexec));
        if (ctx->graph) HIPCHK(hipGraphDestroy(ctx->graph));
        ctx->gexec = nullptr;
        ctx->graph = nullptr;
        return DFT_OK;
    });
}

dft_status dft_destroy(dft_ctx *ctx) {
    if (!ctx) return DFT_OK;
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return DFT_OK;
}

}  // extern "C"
