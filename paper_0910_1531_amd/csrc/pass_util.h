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
__device__ __forceinline__ XFwdArgs shift(XFwdArgs a, long long o) {
    a.src = shp(a.src, o); a.g0 = shp(a.g0, o); a.alpha = shp(a.alpha, o); a.rho_t = shp(a.rho_t, o);
    a.ref = shp(a.ref, o); a.spec = shp(a.spec, o); a.gate = shp(a.gate, o);
    return a;
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
    return a;
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
// Pointwise work of X2 at one real node idx (of N): the ten weighted densities n in
// (FP32-mixed: differences from the reference nref), dPhi/dn of eq. (Phi) out in d
// (FP32-mixed: the difference from dPhi/dn at the reference; X2_HESS: the product
// Phi''(nstar) n).  Updates the running maximum of n3 and the flags (1: the evaluation is
// non-finite, 2: xi^2 clamped, 4: n3 itself non-finite) and writes the optional FP64 /
// FP32 copies.
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
        fmt_dphi<Dual>(nd, dd, clamped);
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
        fmt_dphi<double>(n, d, clamped);
        fmt_dphi<double>(nr, dr, c2);
#pragma unroll
        for (int f = 0; f < DFT_NALPHA; ++f) d[f] -= dr[f];
    } else {
        fmt_dphi<double>(n, d, clamped);
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

}  // namespace dft
