// Launchers of the compiled-length x passes (X1, X2, X3).
#include "ct_kernels.h"

namespace dft {

// Lengths whose x2 runs the paired-wave kernel k_x2p (wave-private tiles of four values per thread):
// FP32 differences from the reference without FP64 copies, and FP64 in every mode but the n3-only.
template <int L>
constexpr bool x2_paired() { return L == 16 || L == 64 || L == 256; }

// Launches the pass; returns the number of blocks (each writes one n3-maximum partial).
template <typename T, int L>
static int launch_x2c_len(const Geo &g, const X2Args &a, hipStream_t s) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    const long long nb = ct_cdiv(npairs, XTile<L>::PB);
    if (nb > a.red.cap) throw std::runtime_error("x2: reduction buffer too small");
    const dim3 grid((unsigned)nb, 1, (unsigned)g.nprob);
    if (a.hs != DFT_HS_RSLT && a.mode != X2_N3_ONLY) {
        // other functionals: FP64 nodewise work, kernels of their own (launch_x2_alt_ct)
        if (!launch_x2_alt_ct<T>(g, a, s)) throw std::runtime_error("x2: no kernel for this functional");
        return (int)nb;
    }
    constexpr bool fp32 = std::is_same<T, float>::value;
    // FP32: differences from the reference with no FP64 copies requested (FP32 nodewise work)
    const bool d32 = fp32 && a.mode == X2_FULL && a.nref && !a.n_out && !a.dphi_out && !a.nref_out;
    if constexpr (x2_paired<L>()) {
        if (fp32 ? d32 : a.mode != X2_N3_ONLY) {
            const long long nbp = ct_cdiv(npairs, XPairTile<T, L>::PB);
            if (nbp > a.red.cap) throw std::runtime_error("x2: reduction buffer too small");
            hipLaunchKernelGGL((k_x2p<T, L>), dim3((unsigned)nbp, 1, (unsigned)g.nprob), dim3(XPairTile<T, L>::NTB), 0,
                               s, g, a);
            ct_check("x2 paired (compiled length)");
            return (int)nbp;
        }
    } else if constexpr (fp32) {
        if (d32) {
            hipLaunchKernelGGL((k_x2c<T, L, X2N_D32>), grid, dim3(XTile<L>::NTB), 0, s, g, a);
            ct_check("x2 (compiled length)");
            return (int)nb;
        }
    }
    hipLaunchKernelGGL((k_x2c<T, L, X2N_FP64>), grid, dim3(XTile<L>::NTB), 0, s, g, a);
    ct_check("x2 (compiled length)");
    return (int)nb;
}

template <typename T, int L>
static void launch_x1c_len(const Geo &g, const XFwdArgs &a, hipStream_t s) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    dim3 grid((unsigned)ct_cdiv(npairs, XTile<L>::PB), (unsigned)a.nfield, (unsigned)g.nprob);
    hipLaunchKernelGGL((k_x1c<T, L>), grid, dim3(XTile<L>::NTB), 0, s, g, a);
    ct_check("x1 (compiled length)");
}

template <typename T, int L>
static void launch_x3c_len(const Geo &g, const X3Args &a, hipStream_t s) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    const long long nb = ct_cdiv(npairs, XTile<L>::PB);
    if (!a.raw && nb * a.nfield > a.red.cap) throw std::runtime_error("x3: reduction buffer too small");
    dim3 grid((unsigned)nb, (unsigned)a.nfield, (unsigned)g.nprob);
    hipLaunchKernelGGL((k_x3c<T, L>), grid, dim3(XTile<L>::NTB), 0, s, g, a);
    ct_check("x3 (compiled length)");
}

template <typename T>
int launch_x2_ct(const Geo &g, const X2Args &a, hipStream_t s) {
    switch (g.nx) {
#define DFT_CASE(n) case n: return launch_x2c_len<T, n>(g, a, s);
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return 0;
    }
}

template <typename T>
bool launch_x1_ct(const Geo &g, const XFwdArgs &a, hipStream_t s) {
    switch (g.nx) {
#define DFT_CASE(n) case n: launch_x1c_len<T, n>(g, a, s); return true;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

template <typename T>
bool launch_x3_ct(const Geo &g, const X3Args &a, hipStream_t s) {
    switch (g.nx) {
#define DFT_CASE(n) case n: launch_x3c_len<T, n>(g, a, s); return true;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

// Row pairs per block of the compiled-length x kernels (0: the length has none).
int x_ct_pairs(int nx) {
    switch (nx) {
#define DFT_CASE(n) case n: return XTile<n>::PB;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return 0;
    }
}

// Fewest row pairs per block of any compiled-length x2 kernel of the length (paired tiles hold
// half as many as the others): bounds the number of n3-maximum partials.
int x2_ct_min_pairs(int nx) {
    switch (nx) {
#define DFT_CASE(n) case n: return x2_paired<n>() ? XPairTile<float, n>::PB : XTile<n>::PB;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return 0;
    }
}

template bool launch_x1_ct<double>(const Geo &, const XFwdArgs &, hipStream_t);
template bool launch_x1_ct<float>(const Geo &, const XFwdArgs &, hipStream_t);
template int launch_x2_ct<double>(const Geo &, const X2Args &, hipStream_t);
template int launch_x2_ct<float>(const Geo &, const X2Args &, hipStream_t);
template bool launch_x3_ct<double>(const Geo &, const X3Args &, hipStream_t);
template bool launch_x3_ct<float>(const Geo &, const X3Args &, hipStream_t);

}  // namespace dft
