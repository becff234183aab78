// Launchers of the compiled-length Z2 pass, with the tile widths the autotuner chooses
// among.
#include "ct_kernels.h"

namespace dft {

template <typename T> constexpr int z2_width(int v);
template <> constexpr int z2_width<float>(int v) { return v == 0 ? 8 : 4; }
template <> constexpr int z2_width<double>(int v) { return v == 0 ? 4 : 2; }

template <typename T, int L, int V>
static void launch_z2c_var(const Geo &g, const Z2Args &a, hipStream_t s) {
    constexpr int P = z2_width<T>(V), NTB = fit_threads(L, P, 4, 512);
    dim3 grid((unsigned)ct_cdiv(g.Kx, P), (unsigned)g.ny, (unsigned)g.nprob);
    hipLaunchKernelGGL((k_z2c<T, L, P, NTB>), grid, dim3(NTB), 0, s, g, a);
    ct_check("z2 (compiled length)");
}

template <typename T>
bool launch_z2_ct(const Geo &g, const Z2Args &a, hipStream_t s) {
    const int v = g.tune[TUNE_Z2][std::is_same<T, float>::value ? 1 : 0];
    switch (g.nz) {
#define DFT_CASE(n) \
    case n: if (v == 1) launch_z2c_var<T, n, 1>(g, a, s); else launch_z2c_var<T, n, 0>(g, a, s); return true;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

// Number of z shapes for a length (0: no compiled kernel).
int z_ct_variants(int L) {
    switch (L) {
#define DFT_CASE(n) case n: return 2;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return 0;
    }
}

template bool launch_z2_ct<double>(const Geo &, const Z2Args &, hipStream_t);
template bool launch_z2_ct<float>(const Geo &, const Z2Args &, hipStream_t);

}  // namespace dft
