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
// Geometry of problem `prob`: its constants move with its workspace; twiddles are shared.
__device__ __forceinline__ Geo shift(Geo g, long long o) {
    g.cs = shp(g.cs, o);
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

}  // namespace dft
