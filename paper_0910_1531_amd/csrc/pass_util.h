// Device helpers shared by the pass kernels: twiddle tables, gates, batch pointer
// shifts and the XCD-aware block order.
#pragma once

#include <type_traits>

#include "dft_kernels.h"

namespace dft {

// Twiddle table of one axis.  The axis is selected with constant indices so that the
// kernel argument block is never copied to scratch memory for a run-time array index.
template <typename T> __device__ __forceinline__ const cx<T> *twp(const Geo &g, int axis);
template <> __device__ __forceinline__ const cx<double> *twp<double>(const Geo &g, int axis) {
    const void *t = axis == 0 ? g.tw64[0] : axis == 1 ? g.tw64[1] : g.tw64[2];
    return reinterpret_cast<const cx<double> *>(t);
}
template <> __device__ __forceinline__ const cx<float> *twp<float>(const Geo &g, int axis) {
    const void *t = axis == 0 ? g.tw32[0] : axis == 1 ? g.tw32[1] : g.tw32[2];
    return reinterpret_cast<const cx<float> *>(t);
}

__device__ __forceinline__ bool gated_off(const int *gate) { return gate != nullptr && *gate == 0; }

// ------------------------------------------------------------------ batches
// Pointers of problem `prob` of a batch: every workspace pointer moves by prob * pstride.
template <typename P>
__device__ __forceinline__ P *shp(P *ptr, long long off) {
    return ptr ? reinterpret_cast<P *>(reinterpret_cast<char *>(const_cast<typename std::remove_const<P>::type *>(ptr)) + off)
               : nullptr;
}
__device__ __forceinline__ RedBufs shift(RedBufs r, long long o) {
    r.fpart = shp(r.fpart, o); r.mpart = shp(r.mpart, o); r.fflag = shp(r.fflag, o); r.mflag = shp(r.mflag, o);
    return r;
}
__device__ __forceinline__ Roles shift(Roles r, long long o) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r.rho[k] = shp(r.rho[k], o);
        r.G[k] = shp(r.G[k], o);
    }
    r.sel = shp(r.sel, o);
    return r;
}
__device__ __forceinline__ XFwdArgs shift(XFwdArgs a, long long o) {
    a.src = shp(a.src, o); a.g0 = shp(a.g0, o); a.alpha = shp(a.alpha, o); a.rho_t = shp(a.rho_t, o);
    a.ref = shp(a.ref, o); a.spec = shp(a.spec, o); a.gate = shp(a.gate, o); a.roles = shift(a.roles, o);
    return a;
}
// Entry k of a role table, chosen by selects (a run-time index into the argument array would
// put the arguments in scratch memory); k is uniform over the launch.
template <typename P>
__device__ __forceinline__ P *role_pick(P *const (&t)[4], int k) {
    return k == 0 ? t[0] : (k == 1 ? t[1] : (k == 2 ? t[2] : t[3]));
}
// The problem's current role, read once per wave into a scalar register.
__device__ __forceinline__ int role_sel(const int *sel) { return __builtin_amdgcn_readfirstlane(*sel) & 3; }

// The buffers of a line-search pass from the problem's roles (after shift, past the gate).
__device__ __forceinline__ void resolve_roles(XFwdArgs &a) {
    if (!a.roles.sel) return;
    const int s = role_sel(a.roles.sel);
    a.src = role_pick(a.roles.rho, s);
    if (a.kind == ROLE_PRIME) {
        a.g0 = role_pick(a.roles.rho, s);
        a.rho_t = nullptr;
    } else {
        a.g0 = role_pick(a.roles.G, s);
        a.rho_t = a.kind == ROLE_N3 ? nullptr : role_pick(a.roles.rho, (s + 1 + a.kind) & 3);
    }
}
__device__ __forceinline__ YArgs shift(YArgs a, long long o) {
    a.spec = shp(a.spec, o); a.gate = shp(a.gate, o);
    return a;
}
__device__ __forceinline__ Z1Args shift(Z1Args a, long long o) {
    a.specA = shp(a.specA, o); a.specB = shp(a.specB, o); a.gate = shp(a.gate, o);
    return a;
}
__device__ __forceinline__ Z2Args shift(Z2Args a, long long o) {
    a.specA = shp(a.specA, o); a.specB = shp(a.specB, o); a.gate = shp(a.gate, o);
    return a;
}
__device__ __forceinline__ X2Args shift(X2Args a, long long o) {
    a.specB = shp(a.specB, o); a.nref = shp(a.nref, o); a.nref_out = shp(a.nref_out, o);
    a.n_out = shp(a.n_out, o); a.dphi_out = shp(a.dphi_out, o); a.nstar = shp(a.nstar, o);
    a.t_out = shp(a.t_out, o); a.red = shift(a.red, o); a.gate = shp(a.gate, o);
    return a;
}
__device__ __forceinline__ X3Args shift(X3Args a, long long o) {
    a.specA = shp(a.specA, o); a.addend = shp(a.addend, o); a.raw_out = shp(a.raw_out, o);
    a.base = shp(a.base, o); a.rho_t = shp(a.rho_t, o); a.g_out = shp(a.g_out, o); a.e_out = shp(a.e_out, o);
    a.e_phi = shp(a.e_phi, o); a.lp_out = shp(a.lp_out, o); a.red = shift(a.red, o); a.gate = shp(a.gate, o);
    a.roles = shift(a.roles, o);
    return a;
}
__device__ __forceinline__ void resolve_roles(X3Args &a) {
    if (!a.roles.sel) return;
    const int s = role_sel(a.roles.sel);
    const int t = a.kind == ROLE_PRIME ? s : (s + 1 + a.kind) & 3;
    a.rho_t = role_pick(a.roles.rho, t);
    a.g_out = role_pick(a.roles.G, t);
}
// Geometry of problem `prob`: its constants and spectral tables move with its workspace;
// twiddles are shared.
__device__ __forceinline__ Geo shift(Geo g, long long o) {
    g.cs = shp(g.cs, o);
    g.tab64 = shp(g.tab64, o);
    return g;
}

// Block coordinates with consecutive column chunks kept on one XCD: blocks are dispatched
// round-robin over the 8 XCDs by linear id, so linear ids are regrouped into 8 contiguous
// runs (when the grid divides evenly) and neighbouring chunks share an L2.
__device__ __forceinline__ void xcd_block(int &bx, int &by) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int B = gx * gy;
    int l = blockIdx.x + gx * blockIdx.y;
    if ((B & 7) == 0) l = (l & 7) * (B >> 3) + (l >> 3);
    bx = l % gx;
    by = l / gx;
}

// ------------------------------------------------------------------ block reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_down(v, o, 64);
    return v;
}

// Fixed-order block reduction (sum or max) of one double and an OR of one int.
template <bool MAX, int NTB>
__device__ __forceinline__ void block_reduce_nt(double v, int fl, double *dst, int *fdst) {
    __shared__ double sv[NTB / 64];
    __shared__ int sf[NTB / 64];
    v = MAX ? wave_max(v) : wave_sum(v);
    fl = wave_or(fl);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) { sv[w] = v; sf[w] = fl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = sv[0];
        int f = sf[0];
        for (int i = 1; i < NTB / 64; ++i) { a = MAX ? fmax(a, sv[i]) : a + sv[i]; f |= sf[i]; }
        *dst = a;
        *fdst = f;
    }
}

// ------------------------------------------------------------------ X2 node work
// Pointwise work of X2 at one real node idx (of N), for eq. (Phi) (ALT = false) or the
// alternative functional a.hs (ALT = true): the ten weighted densities n in
// (FP32-mixed: differences from the reference nref), dPhi/dn of eq. (Phi) out in d
// (FP32-mixed: the difference from dPhi/dn at the reference; X2_HESS: the product
// Phi''(nstar) n).  Updates the running maximum of n3 and the flags (1: the evaluation is
// non-finite, 2: xi^2 clamped, 4: n3 itself non-finite) and writes the optional FP64 /
// FP32 copies.
template <bool ALT>
__device__ __forceinline__ void x2_node(const X2Args &a, long long N, long long idx, const double (&nin)[DFT_NALPHA],
                                        double (&d)[DFT_NALPHA], double &mloc, int &flag) {
    double n[DFT_NALPHA];
#pragma unroll
    for (int f = 0; f < DFT_NALPHA; ++f) n[f] = nin[f];
    bool clamped = false;
    if (a.mode == X2_HESS) {
        Dual nd[DFT_NALPHA], dd[DFT_NALPHA];
#pragma unroll
        for (int f = 0; f < DFT_NALPHA; ++f) nd[f] = Dual{a.nstar[f * N + idx], n[f]};
        fmt_dphi_as<ALT, Dual>(a.hs, nd, dd, clamped);
        bool bad = false;
#pragma unroll
        for (int f = 0; f < DFT_NALPHA; ++f) {
            d[f] = dd[f].d;
            bad |= !isfinite(d[f]);
            if (a.t_out) a.t_out[f * N + idx] = d[f];
        }
        if (bad) flag |= 1;
        return;
    }
    if (a.nref) {
        double nr[DFT_NALPHA], dr[DFT_NALPHA];
#pragma unroll
        for (int f = 0; f < DFT_NALPHA; ++f) {
            nr[f] = (double)a.nref[f * N + idx];
            n[f] += nr[f];
        }
        bool c2;
        fmt_dphi_as<ALT, double>(a.hs, n, d, clamped);
        fmt_dphi_as<ALT, double>(a.hs, nr, dr, c2);
#pragma unroll
        for (int f = 0; f < DFT_NALPHA; ++f) d[f] -= dr[f];
    } else {
        fmt_dphi_as<ALT, double>(a.hs, n, d, clamped);
    }
    if (clamped) flag |= 2;
    if (!isfinite(n[3])) flag |= 5;                        // 1: evaluation non-finite, 4: n3 non-finite
    if (!isfinite(d[0]) || !isfinite(d[3])) flag |= 1;     // e.g. n3 >= 1: f = +inf, n3 max still valid
    mloc = fmax(mloc, n[3]);
#pragma unroll
    for (int f = 0; f < DFT_NALPHA; ++f) {
        if (a.nref_out) a.nref_out[f * N + idx] = (float)n[f];
        if (a.n_out) a.n_out[f * N + idx] = n[f];
        if (a.dphi_out) a.dphi_out[f * N + idx] = d[f];
    }
}

// FP64 reciprocal: the hardware estimate refined by one Newton step (error about 1 ulp of FP64).
__device__ __forceinline__ double rcp64(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// log(1 + u) in FP64.  For |u| <= 1/4, 2 atanh(s) with s = u / (2 + u) (|s| <= 1/7) summed to s^21,
// which is below an FP64 ulp of the result (to s^5 when |s| < 2^-10: the next term is below
// 2^-60 of s); otherwise the library's log1p.
__device__ __forceinline__ double log1p64(double u) {
    if (!(fabs(u) <= 0.25)) return log1p(u);
    const double s = u * rcp64(2.0 + u), s2 = s * s;
    if (fabs(s) < 0x1p-10) return 2.0 * fma(s * s2, fma(s2, 1.0 / 5.0, 1.0 / 3.0), s);
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    return 2.0 * fma(s * s2, p, s);
}

// FP32-mixed nodewise work of X2: the difference dPhi(nr + dn) - dPhi(nr) of eq. (Phi).  The
// factors that carry the packing singularity -- log(1 - n3) and the powers 1 / (1 - n3)^k with
// their differences from the reference -- are formed in FP64 from the FP32 inputs; the rest in
// FP32 term by term.  Every product is expanded by telescoping, a b - ar br = (a - ar) b +
// ar (b - br), and every term carries one difference factor, so the rounding error is
// proportional to |dn|, as in the FP32 transforms; log(1 - n3) enters only as
// log1p(-dn3 / (1 - nr3)).  The FP32 reciprocals (the xi^2 ratio) use the hardware's reciprocal
// instruction (about 1 ulp; the coefficients need FP32 relative accuracy only).  n3 itself (the
// line-search bound) is formed in FP64.  Flags and the n3 maximum as x2_node.
// nrv holds the reference values nref[f][idx], loaded by the caller ahead of time.
__device__ __forceinline__ void x2_node_diff(const float (&nrv)[DFT_NALPHA], const float (&dn)[DFT_NALPHA],
                                             float (&dd)[DFT_NALPHA], double &mloc, int &flag) {
    float nr[DFT_NALPHA], n[DFT_NALPHA];
#pragma unroll
    for (int f = 0; f < DFT_NALPHA; ++f) {
        nr[f] = nrv[f];
        n[f] = nr[f] + dn[f];
    }
    const double n3 = (double)nr[3] + (double)dn[3];
    const float inv8pi = (float)(1.0 / (8.0 * 3.14159265358979323846));
    const float inv12pi = (float)(1.0 / (12.0 * 3.14159265358979323846));
    const float inv4pi = (float)(1.0 / (4.0 * 3.14159265358979323846));
    // 1 / (1 - n3) and its powers, with their differences (FP64, rounded once to FP32)
    const double dn3 = (double)dn[3];
    const double Drd = 1.0 - (double)nr[3], Dd = Drd - dn3;
    const double iDrd = rcp64(Drd), iDd = rcp64(Dd);
    const double diDd = dn3 * iDd * iDrd;
    const float iD = (float)iDd, diD = (float)diDd;
    const float iD2 = (float)(iDd * iDd), diD2 = (float)(diDd * (iDd + iDrd));
    const float iD3 = (float)(iDd * iDd * iDd), diD3 = (float)(diDd * (iDd * iDd + iDd * iDrd + iDrd * iDrd));
    // vector products and the xi^2 = nV2.nV2 / n2^2 ratio, clamped at 1
    float dot12r = 0.f, ddot12 = 0.f, dot22 = 0.f, dot22r = 0.f, ddot22 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dot12r += nr[4 + d] * nr[7 + d];
        ddot12 += dn[4 + d] * n[7 + d] + nr[4 + d] * dn[7 + d];
        dot22 += n[7 + d] * n[7 + d];
        dot22r += nr[7 + d] * nr[7 + d];
        ddot22 += dn[7 + d] * (n[7 + d] + nr[7 + d]);
    }
    const float tiny = 1e-30f;
    const float n2sq = n[2] * n[2], n2sqr = nr[2] * nr[2], dn2sq = dn[2] * (n[2] + nr[2]);
    const float den = fmaxf(n2sq, tiny), denr = fmaxf(n2sqr, tiny);
    const float dden = (n2sq > tiny && n2sqr > tiny) ? dn2sq : den - denr;
    const float x2 = dot22 * rcp_r(den), x2r = dot22r * rcp_r(denr);
    float dxc;
    // x2 - x2r = (d(dot22) - x2r d(den)) / den: no product of two floored denominators, which
    // underflows where n2 vanishes
    if (x2 < 1.0f && x2r < 1.0f) dxc = (ddot22 - x2r * dden) * rcp_r(den);
    else if (!(x2 < 1.0f) && !(x2r < 1.0f)) dxc = 0.0f;
    else dxc = fminf(x2, 1.0f) - fminf(x2r, 1.0f);
    const float xc = fminf(x2, 1.0f), xcr = fminf(x2r, 1.0f);
    const float q = 1.0f - xc, qr = 1.0f - xcr, dq = -dxc;
    const float q2 = q * q, q2r = qr * qr, dq2 = dq * (q + qr);
    const float q3 = q2 * q, q3r = q2r * qr, dq3 = dq * (q2 + q * qr + q2r);
    if (!(x2 < 1.0f)) flag |= 2;
    // d0 = -log(1 - n3) + log(1 - nr3)
    dd[0] = (float)(-log1p64(-dn3 * iDrd));
    // d1 = n2 / D
    dd[1] = dn[2] * iD + nr[2] * diD;
    // d2 = n1 / D + n2^2 q^2 (1 + xi^2) / (8 pi D^2)
    {
        const float t1 = dn[1] * iD + nr[1] * diD;
        const float C = 1.0f + xc, Cr = 1.0f + xcr;
        const float t2 = dn2sq * q2 * C * iD2 + n2sqr * dq2 * C * iD2 + n2sqr * q2r * dxc * iD2 +
                         n2sqr * q2r * Cr * diD2;
        dd[2] = t1 + t2 * inv8pi;
    }
    // d3 = n0 / D + (n1 n2 - nV1.nV2) / D^2 + n2^3 q^3 / (12 pi D^3)
    {
        const float t1 = dn[0] * iD + nr[0] * diD;
        const float Mr = nr[1] * nr[2] - dot12r;
        const float dM = dn[1] * n[2] + nr[1] * dn[2] - ddot12;
        const float t2 = dM * iD2 + Mr * diD2;
        const float n2cr = n2sqr * nr[2];
        const float dn2c = dn[2] * (n2sq + n[2] * nr[2] + n2sqr);
        const float t3 = dn2c * q3 * iD3 + n2cr * dq3 * iD3 + n2cr * q3r * diD3;
        dd[3] = t1 + t2 + t3 * inv12pi;
    }
    // d4..6 = -nV2 / D;  d7..9 = -nV1 / D - n2 q^2 nV2 / (4 pi D^2)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dd[4 + d] = -(dn[7 + d] * iD + nr[7 + d] * diD);
        const float t1 = dn[4 + d] * iD + nr[4 + d] * diD;
        const float t2 = dn[2] * q2 * n[7 + d] * iD2 + nr[2] * dq2 * n[7 + d] * iD2 +
                         nr[2] * q2r * dn[7 + d] * iD2 + nr[2] * q2r * nr[7 + d] * diD2;
        dd[7 + d] = -t1 - t2 * inv4pi;
    }
    if (!isfinite(n3)) flag |= 5;                           // 1: evaluation non-finite, 4: n3 non-finite
    if (!isfinite(dd[0]) || !isfinite(dd[3]) || !(Dd > 0.0)) flag |= 1;
    mloc = fmax(mloc, n3);
}

}  // namespace dft
