// Launchers of the compiled-length y passes (and plain z transforms), with the launch
// shapes the autotuner chooses among: P adjacent columns per tile (P complex values are
// contiguous in HBM), threads per tile and one or two LDS exchange buffers.
#include "ct_kernels.h"

namespace dft {

// Shape v of the y kernel for precision T: tile width, values per thread (8, or 16 for shapes
// 3 and 4: half the threads, two butterflies per thread and stage) and LDS buffers (shapes 5-9:
// shapes 0-4 with one buffer, so more tiles fit per CU at a second barrier per exchange).
template <typename T> constexpr int y_width(int v);
template <> constexpr int y_width<float>(int v) {
    return (v % 5 == 0 || v % 5 == 3) ? 16 : (v % 5 == 1 || v % 5 == 4) ? 8 : 32;
}
template <> constexpr int y_width<double>(int v) {
    return (v % 5 == 0 || v % 5 == 3) ? 8 : (v % 5 == 1 || v % 5 == 4) ? 4 : 16;
}
constexpr int y_per_thread(int v) { return v % 5 >= 3 ? 16 : 8; }
constexpr int kYVariants = 10;
constexpr int kLdsCap = 65536;

// LDS buffers of shape v (T, L, P): 2 when two tiles fit and the shape asks for two, else 1, 0
// when not even one tile does.
template <typename T, int L, int P, int V>
constexpr int y_buffers() {
    constexpr int tile = L * P * (int)sizeof(cx<T>);
    return (V < 5 && 2 * tile <= kLdsCap) ? 2 : (tile <= kLdsCap ? 1 : 0);
}

template <typename T, int L, int V>
static bool launch_yc_var(const Geo &g, const YArgs &a, hipStream_t s) {
    constexpr int P = y_width<T>(V);
    constexpr int NB = y_buffers<T, L, P, V>();
    if constexpr (NB == 0) {
        return false;
    } else {
        constexpr int NTB = fit_threads(L, P, y_per_thread(V), 256);
        const bool zax = a.axis == 2;
        const int ntypes = a.vec == 1 ? 7 : (a.vec == 2 ? 8 : a.nfield);
        if (zax && a.vec != 0) return false;   // the compact vector layout has y passes only
        // tiles over the flattened plane of pencils: (y, kx) for the z axis, (z, kx) for the y axis
        dim3 grid((unsigned)ct_cdiv((zax ? g.ny : g.nz) * g.Kx, P), 1, (unsigned)(ntypes * g.nprob));
        if (a.vec == 1)
            hipLaunchKernelGGL((k_yc<T, L, P, NTB, NB, 1>), grid, dim3(NTB), 0, s, g, a);
        else if (a.vec == 2)
            hipLaunchKernelGGL((k_yc<T, L, P, NTB, NB, 2>), grid, dim3(NTB), 0, s, g, a);
        else
            hipLaunchKernelGGL((k_yc<T, L, P, NTB, NB, 0>), grid, dim3(NTB), 0, s, g, a);
        ct_check("y (compiled length)");
        return true;
    }
}

template <typename T, int L>
static bool launch_yc_len(const Geo &g, const YArgs &a, hipStream_t s, int v) {
    switch (v) {
        case 1: if (launch_yc_var<T, L, 1>(g, a, s)) return true; break;
        case 2: if (launch_yc_var<T, L, 2>(g, a, s)) return true; break;
        case 3: if (launch_yc_var<T, L, 3>(g, a, s)) return true; break;
        case 4: if (launch_yc_var<T, L, 4>(g, a, s)) return true; break;
        case 5: if (launch_yc_var<T, L, 5>(g, a, s)) return true; break;
        case 6: if (launch_yc_var<T, L, 6>(g, a, s)) return true; break;
        case 7: if (launch_yc_var<T, L, 7>(g, a, s)) return true; break;
        case 8: if (launch_yc_var<T, L, 8>(g, a, s)) return true; break;
        case 9: if (launch_yc_var<T, L, 9>(g, a, s)) return true; break;
        default: break;
    }
    return launch_yc_var<T, L, 0>(g, a, s);
}

template <typename T>
bool launch_y_ct(const Geo &g, const YArgs &a, hipStream_t s) {
    // the ten weighted-density / derivative spectra (compact or not) or the species spectra
    const bool ten = a.vec != 0 || a.nfield == DFT_NALPHA;
    const int pass = a.axis == 2 ? TUNE_YZ : (ten ? (a.dir > 0 ? TUNE_Y : TUNE_YF) : TUNE_YS);
    const int v = g.tune[pass][std::is_same<T, float>::value ? 1 : 0];
    switch (a.axis == 2 ? g.nz : g.ny) {
#define DFT_CASE(n) case n: return launch_yc_len<T, n>(g, a, s, v);
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

// Number of y shapes for a length (0: no compiled kernel).  A shape whose tile does not
// fit the LDS runs as shape 0.
int y_ct_variants(int L, bool) {
    switch (L) {
#define DFT_CASE(n) case n: return kYVariants;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return 0;
    }
}

template bool launch_y_ct<double>(const Geo &, const YArgs &, hipStream_t);
template bool launch_y_ct<float>(const Geo &, const YArgs &, hipStream_t);

}  // namespace dft
