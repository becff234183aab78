// Launchers of the compiled-length Z2 pass, with the tile widths the autotuner chooses
// among.
#include "ct_kernels.h"

namespace dft {

// Spectral tables (FP64) of the z kernels: one thread per half-spectrum element.
__global__ __launch_bounds__(256) void k_spec_tables(Geo g) {
    const long long NC = g.NC;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= NC) return;
    const Consts &c = *g.cs;
    const int Kx = g.Kx, S = g.S;
    const int kx = (int)(i % Kx);
    const long long t = i / Kx;
    const int y = (int)(t % g.ny), e = (int)(t / g.ny);
    const ZWave<double> kw(c, kx, y);
    const double kmag = kw.kmag(e);
    double *t64 = const_cast<double *>(g.tab64);
    auto put = [&](int row, double v) { ct::gst(t64 + (long long)row * NC + i, v); };
    for (int s = 0; s < S; ++s) {
        double w2, w3;
        weight_w2_w3<double>(kmag, c.R[s], w2, w3);
        put(s, w2);
        put(S + s, w3);
    }
    if (g.ntab > 2 * S) {
        double invD = 0.0;
        if (!kw.zero(e)) {
            const Poisson<double> pd(g, c, kx, y);
            invD = c.four_pi_lB / pd.denom(e);
        }
        for (int a = 0; a < S; ++a)
            for (int b = a; b < S; ++b) {
                const int ij = a * DFT_MAX_SPECIES + b;
                const double C = screening_hat<double>(kmag, c.sc_R[ij], c.sc_c1[ij], c.sc_c0[ij], c.sc_cm1[ij]);
                put(pair_row(S, a, b), C - invD * c.z[a] * c.z[b]);
            }
    }
}


template <typename T> constexpr int z2_width(int v);
template <> constexpr int z2_width<float>(int v) { return v == 0 ? 8 : v == 1 ? 4 : 16; }
template <> constexpr int z2_width<double>(int v) { return v == 0 ? 4 : v == 1 ? 2 : 8; }

template <typename T, int L, int V>
static void launch_z2c_var(const Geo &g, const Z2Args &a, hipStream_t s) {
    constexpr int P = z2_width<T>(V), NTB = fit_threads(L, P, 4, 512);
    dim3 grid((unsigned)ct_cdiv(g.ny * g.Kx, P), 1, (unsigned)g.nprob);   // flattened (y, kx) columns
    hipLaunchKernelGGL((k_z2c<T, L, P, NTB>), grid, dim3(NTB), 0, s, g, a);
    ct_check("z2 (compiled length)");
}

template <typename T>
bool launch_z2_ct(const Geo &g, const Z2Args &a, hipStream_t s) {
    if (!g.tab64) return false;   // no spectral tables: run-time-length kernel
    const int v = g.tune[TUNE_Z2][std::is_same<T, float>::value ? 1 : 0];
    switch (g.nz) {
#define DFT_CASE(n)                                  \
    case n:                                          \
        if (v == 1) launch_z2c_var<T, n, 1>(g, a, s);    \
        else if (v == 2) launch_z2c_var<T, n, 2>(g, a, s); \
        else launch_z2c_var<T, n, 0>(g, a, s);           \
        return true;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

// Number of z shapes for a length (0: no compiled kernel).
int z_ct_variants(int L) {
    switch (L) {
#define DFT_CASE(n) case n: return 3;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return 0;
    }
}

// Z1 shapes: the three fused tile widths, then the same widths split into the plain z pass and
// k_z1s.
int z1_ct_variants(int L) { return 2 * z_ct_variants(L); }

int spec_table_rows(int nz, int S, int es) {
    if (z_ct_variants(nz) == 0) return 0;
    if (es && S > 4) return 0;   // electrostatic sums of more species: run-time-length kernels
    return 2 * S + (es ? S * (S + 1) / 2 : 0);
}

void launch_spec_tables(const Geo &g, hipStream_t s) {
    hipLaunchKernelGGL(k_spec_tables, dim3((unsigned)ct_cdiv(g.NC, 256)), dim3(256), 0, s, g);
    ct_check("spectral tables");
}

template bool launch_z2_ct<double>(const Geo &, const Z2Args &, hipStream_t);
template bool launch_z2_ct<float>(const Geo &, const Z2Args &, hipStream_t);

}  // namespace dft
