// Launchers of the compiled-length X2 pass for the alternative hard-sphere functionals
// (Rosenfeld's original vector form, White Bear): FP64 nodewise work in kernels of their own,
// so the kernels of eq. (Phi) keep their register budget.
#include "ct_kernels.h"

namespace dft {

template <typename T, int L>
static void launch_x2c_alt_len(const Geo &g, const X2Args &a, hipStream_t s) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    const long long nb = ct_cdiv(npairs, XTile<L>::PB);
    if (nb > a.red.cap) throw std::runtime_error("x2: reduction buffer too small");
    const dim3 grid((unsigned)nb, 1, (unsigned)g.nprob);
    hipLaunchKernelGGL((k_x2c<T, L, X2N_ALT>), grid, dim3(XTile<L>::NTB), 0, s, g, a);
    ct_check("x2 (compiled length, alternative functional)");
}

template <typename T>
bool launch_x2_alt_ct(const Geo &g, const X2Args &a, hipStream_t s) {
    switch (g.nx) {
#define DFT_CASE(n) case n: launch_x2c_alt_len<T, n>(g, a, s); return true;
        DFT_CT_LENGTHS(DFT_CASE)
#undef DFT_CASE
        default: return false;
    }
}

template bool launch_x2_alt_ct<double>(const Geo &, const X2Args &, hipStream_t);
template bool launch_x2_alt_ct<float>(const Geo &, const X2Args &, hipStream_t);

}  // namespace dft
