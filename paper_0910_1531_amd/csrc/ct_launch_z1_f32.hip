// Launchers of the compiled-length Z1 pass in precision float, with the tile widths the
// autotuner chooses among.
#include "ct_kernels.h"

namespace dft {

template <typename T> constexpr int z_width(int v);
template <> constexpr int z_width<float>(int v) { return v == 0 ? 8 : v == 1 ? 4 : 16; }
template <> constexpr int z_width<double>(int v) { return v == 0 ? 4 : v == 1 ? 2 : 8; }

template <typename T, int L, int V>
static void launch_z1c_var(const Geo &g, const Z1Args &a, int es, hipStream_t s) {
    constexpr int P = z_width<T>(V), NTB = fit_threads(L, P, 4, 512);
    dim3 grid((unsigned)ct_cdiv(g.ny * g.Kx, P), 1, (unsigned)g.nprob);   // flattened (y, kx) columns
    if (!es) hipLaunchKernelGGL((k_z1c<T, L, P, NTB, 0>), grid, dim3(NTB), 0, s, g, a);
    else {
        // the pair accumulators are sized for the species count: fewer registers for S < 4
        if (g.S <= 2) hipLaunchKernelGGL((k_z1c<T, L, P, NTB, 2>), grid, dim3(NTB), 0, s, g, a);
        else if (g.S == 3) hipLaunchKernelGGL((k_z1c<T, L, P, NTB, 3>), grid, dim3(NTB), 0, s, g, a);
        else hipLaunchKernelGGL((k_z1c<T, L, P, NTB, 4>), grid, dim3(NTB), 0, s, g, a);
    }
    ct_check("z1 (compiled length)");
}

// Split shapes (V = 3, 4, 5 for the tile widths of V - 3): the plain z pass transforms the
// species spectra in place, then k_z1s forms the products and the inverse transforms.
template <typename T, int L, int V>
static void launch_z1s_var(const Geo &g, const Z1Args &a, int es, hipStream_t s) {
    YArgs za{a.specA, g.S, -1, a.gate};
    za.axis = 2;
    launch_y<T>(g, za, s);
    constexpr int P = z_width<T>(V), NTB = fit_threads(L, P, 4, 512);
    dim3 grid((unsigned)ct_cdiv(g.ny * g.Kx, P), 1, (unsigned)g.nprob);   // flattened (y, kx) columns
    if (!es) hipLaunchKernelGGL((k_z1s<T, L, P, NTB, 0>), grid, dim3(NTB), 0, s, g, a);
    else if (g.S <= 2) hipLaunchKernelGGL((k_z1s<T, L, P, NTB, 2>), grid, dim3(NTB), 0, s, g, a);
    else if (g.S == 3) hipLaunchKernelGGL((k_z1s<T, L, P, NTB, 3>), grid, dim3(NTB), 0, s, g, a);
    else hipLaunchKernelGGL((k_z1s<T, L, P, NTB, 4>), grid, dim3(NTB), 0, s, g, a);
    ct_check("z1 from z spectra (compiled length)");
}

template <typename T, int L>
static void launch_z1c_len(const Geo &g, const Z1Args &a, int es, hipStream_t s, int v) {
    if (v == 1) launch_z1c_var<T, L, 1>(g, a, es, s);
    else if (v == 2) launch_z1c_var<T, L, 2>(g, a, es, s);
    else if (v == 3) launch_z1s_var<T, L, 0>(g, a, es, s);
    else if (v == 4) launch_z1s_var<T, L, 1>(g, a, es, s);
    else if (v == 5) launch_z1s_var<T, L, 2>(g, a, es, s);
    else launch_z1c_var<T, L, 0>(g, a, es, s);
}

template <>
bool launch_z1_ct<float>(const Geo &g, const Z1Args &a, int es, hipStream_t s) {
    if (!g.tab64) return false;   // no spectral tables (or S > 4 with electrostatics): run-time kernel
    // the on-the-fly pair factors take sin and cos of k (R_i + R_j) by the addition theorem, so a
    // screening cutoff at lambda_i + lambda_j runs the run-time-length kernel
    if (es && g.cut_lambda) return false;
    const int v = g.tune[TUNE_Z1][std::is_same<float, float>::value ? 1 : 0];
    switch (g.nz) {
#define DFT_CASE(n) case n: launch_z1c_len<float, n>(g, a, es, s, v); return true;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

}  // namespace dft
