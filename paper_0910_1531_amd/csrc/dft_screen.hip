// Pointwise kernels of the RFD screening operator (reference-fluid-density section, eqs.
// rhoRef, rhoRefKDotProduct, screening-kernel-hat).  The ball average with a radius R_SC(x) that
// varies in space is not a convolution; the paper applies it as an O(N^2) dot product per grid
// point.  Here the ball transform is interpolated in the radius: the field is convolved (by FFT)
// with the balls of M Chebyshev radii spanning the range of R_SC, and every point combines the M
// results with the barycentric Lagrange weights of its own radius.  These kernels find the
// range, the per-point barycentric denominators and do the weighted accumulation; the
// convolutions run through the transform passes (Z2_BALL).
#include <stdexcept>

#include "dft_screen.h"

namespace dft {

namespace {

constexpr int kNT = 256;

__device__ __forceinline__ void cheb_node(int j, int M, double cc, double dd, double &Rj, double &wj) {
    double sn, cs;
    sincospi((2.0 * j + 1.0) / (2.0 * M), &sn, &cs);
    Rj = cc + dd * cs;
    wj = (j & 1) ? -sn : sn;
}

__global__ __launch_bounds__(kNT) void k_rsc_range(long long n, const double *r, double *pmin, double *pmax,
                                                   int *pbad) {
    __shared__ double smin[kNT], smax[kNT];
    __shared__ int sbad[kNT];
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    for (long long i = (long long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long long)gridDim.x * kNT) {
        const double v = r[i];
        if (!(v > 0.0) || !isfinite(v)) {
            ++bad;
        } else {
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kNT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbad[threadIdx.x] += sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmin[blockIdx.x] = smin[0];
        pmax[blockIdx.x] = smax[0];
        pbad[blockIdx.x] = sbad[0];
    }
}

__global__ __launch_bounds__(kNT) void k_cheb_prep(long long n, const double *r, int M, double cc, double dd,
                                                   double *inv_den, int *hit) {
    const long long x = (long long)blockIdx.x * kNT + threadIdx.x;
    if (x >= n) return;
    const double R = r[x];
    double den = 0.0;
    int h = -1;
    for (int j = 0; j < M; ++j) {
        double Rj, wj;
        cheb_node(j, M, cc, dd, Rj, wj);
        const double t = R - Rj;
        if (t == 0.0) h = j;
        else den += wj / t;
    }
    inv_den[x] = h >= 0 ? 0.0 : 1.0 / den;
    hit[x] = h;
}

__global__ __launch_bounds__(kNT) void k_cheb_accum(long long n, int S, int m, int M, double cc, double dd,
                                                    const double *r, const double *inv_den, const int *hit,
                                                    const double *part, double *out, int first) {
    const long long x = (long long)blockIdx.x * kNT + threadIdx.x;
    if (x >= n) return;
    double Rm, wm;
    cheb_node(m, M, cc, dd, Rm, wm);
    const int h = hit[x];
    const double l = h >= 0 ? (h == m ? 1.0 : 0.0) : wm / (r[x] - Rm) * inv_den[x];
    for (int i = 0; i < S; ++i) {
        const long long o = (long long)i * n + x;
        const double v = l * part[o];
        out[o] = first ? v : out[o] + v;
    }
}

void check(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

long long blocks_for(long long n) { return (n + kNT - 1) / kNT; }

}  // namespace

int rsc_range(long long n, const double *r, double *pmin, double *pmax, int *pbad, int cap, hipStream_t s) {
    long long nb = blocks_for(n);
    if (nb > cap) nb = cap;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_rsc_range, dim3((unsigned)nb), dim3(kNT), 0, s, n, r, pmin, pmax, pbad);
    check("rsc range");
    return (int)nb;
}

void cheb_prep(long long n, const double *r, int M, double cc, double dd, double *inv_den, int *hit, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_prep, dim3((unsigned)blocks_for(n)), dim3(kNT), 0, s, n, r, M, cc, dd, inv_den, hit);
    check("cheb prep");
}

void cheb_accum(long long n, int S, int m, int M, double cc, double dd, const double *r, const double *inv_den,
                const int *hit, const double *part, double *out, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_accum, dim3((unsigned)blocks_for(n)), dim3(kNT), 0, s, n, S, m, M, cc, dd, r, inv_den,
                       hit, part, out, first ? 1 : 0);
    check("cheb accum");
}

}  // namespace dft
