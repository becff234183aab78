// Kernels of the implicit adjoint through the converged fixed point.
//
// With G = rho_b exp(base + E[rho]) on fluid nodes, dG/drho = diag(G) H, H = dE/drho
// (symmetric).  The adjoint weights w = G o lambda solve (diag(G)^-1 - H) w = dO/drho on
// fluid nodes: the grand-potential Hessian, symmetric positive definite at a stable
// solution.  The solve is a conjugate-gradient acceleration of the adjoint Picard
// iteration w <- G o (dO/drho + H w) (preconditioner diag(G)); each iteration applies H
// once through the residual passes with the Hessian-vector FMT kernel.  Parameter
// gradients follow as lambda^T dG/dtheta, the field-dependent parts as spectral
// bilinear sums evaluated here.
#include "dft_adjoint.h"

#include <stdexcept>

namespace dft {

constexpr int NTA = 256;

static void check_launch_a(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// Block partials of up to NV doubles, fixed order: wave sums, then thread 0 over waves.
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *dst) {
    __shared__ double sh[NTA / 64][NV];
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (l == 0) sh[w][k] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = sh[0][k];
            for (int i = 1; i < NTA / 64; ++i) a += sh[i][k];
            dst[k] = a;
        }
    }
}

#define GRID_STRIDE(i, n) for (long long i = (long long)blockIdx.x * NTA + threadIdx.x; i < (n); i += (long long)gridDim.x * NTA)

__global__ __launch_bounds__(NTA) void k_adj_init(long long n, const double *G, const double *g, double *w) {
    GRID_STRIDE(i, n) w[i] = G[i] > 0.0 ? G[i] * g[i] : 0.0;
}

// r = H w on fluid nodes (r0 = g - A w0 for w0 = G o g), p = G o r; partials (r.Gr, r.r)
__global__ __launch_bounds__(NTA) void k_adj_r0(long long n, const double *G, const double *Hw, double *r, double *p,
                                                double *part) {
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, n) {
        const double gi = G[i];
        const double ri = gi > 0.0 ? Hw[i] : 0.0;
        r[i] = ri;
        p[i] = gi * ri;
        v[0] += ri * gi * ri;
        v[1] += ri * ri;
    }
    block_partials<2>(v, part + 2 * blockIdx.x);
}

// q = p / G - H p on fluid nodes; partial p.q
__global__ __launch_bounds__(NTA) void k_adj_q(long long n, const double *G, const double *p, const double *Hp, double *q,
                                               double *part) {
    double v[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double gi = G[i];
        const double qi = gi > 0.0 ? p[i] / gi - Hp[i] : 0.0;
        q[i] = qi;
        v[0] += p[i] * qi;
    }
    block_partials<1>(v, part + blockIdx.x);
}

// w += a p, r -= a q; partials (r.Gr, r.r)
__global__ __launch_bounds__(NTA) void k_adj_step(long long n, double a, const double *G, const double *p, const double *q,
                                                  double *w, double *r, double *part) {
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, n) {
        w[i] += a * p[i];
        const double ri = r[i] - a * q[i];
        r[i] = ri;
        v[0] += ri * G[i] * ri;
        v[1] += ri * ri;
    }
    block_partials<2>(v, part + 2 * blockIdx.x);
}

// p = G o r + b p
__global__ __launch_bounds__(NTA) void k_adj_dir(long long n, double b, const double *G, const double *r, double *p) {
    GRID_STRIDE(i, n) p[i] = G[i] * r[i] + b * p[i];
}

// partial sums of one species' field (blockIdx.y = species)
__global__ __launch_bounds__(NTA) void k_adj_fieldsum(long long N, const double *f, double *part) {
    double v[1] = {0.0};
    const double *fi = f + (long long)blockIdx.y * N;
    GRID_STRIDE(i, N) v[0] += fi[i];
    block_partials<1>(v, part + (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(NTA) void k_adj_neg(long long n, const double *w, double *out) {
    GRID_STRIDE(i, n) out[i] = -w[i];
}

// Newton right-hand side (G - rho) / G on fluid nodes (G > 0), 0 elsewhere.
__global__ __launch_bounds__(NTA) void k_newton_rhs(long long n, const double *G, const double *rho, double *g) {
    GRID_STRIDE(i, n) g[i] = G[i] > 0.0 ? (G[i] - rho[i]) / G[i] : 0.0;
}

// Per-block minimum of -rho / d over nodes with d < 0 (the step that would reach rho = 0).
__global__ __launch_bounds__(NTA) void k_newton_bound(long long n, const double *rho, const double *d, double *part) {
    __shared__ double sh[NTA];
    double m = INFINITY;
    GRID_STRIDE(i, n) {
        if (d[i] < 0.0) m = fmin(m, -rho[i] / d[i]);
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = NTA / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(NTA) void k_axpy(long long n, const double *x, double a, const double *d, double *out) {
    GRID_STRIDE(i, n) out[i] = x[i] + a * d[i];
}

// Sum nparts partial records of width nv into out[0..nv) in a fixed order.
__global__ __launch_bounds__(NTA) void k_adj_reduce(const double *part, int nparts, int nv, double *out) {
    __shared__ double sh[NTA];
    for (int k = 0; k < nv; ++k) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nparts; b += NTA) a += part[(long long)b * nv + k];
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int s = NTA / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = sh[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- spectral sums
// Per species k: j0(kR), cos(kR) and g3 = (sin y - y cos y) / y^3 at y = |k| R.
__device__ __forceinline__ void radial_fns(double kmag, double R, double &j0, double &cy, double &g3) {
    const double y = kmag * R;
    if (y < 1.0) {
        constexpr SincSeries s0{};
        constexpr BallSeries<0> s3{};
        const double y2 = y * y;
        j0 = horner_y2<double>(s0, y2);
        g3 = horner_y2<double>(s3, y2);
        cy = cos(y);
    } else {
        double s, c;
        sincos(y, &s, &c);
        const double iy = 1.0 / y;
        j0 = s * iy;
        cy = c;
        g3 = (s - y * c) * iy * iy * iy;
    }
}

__device__ __forceinline__ double dotc(cx<double> a, cx<double> b) { return a.x * b.x + a.y * b.y; }   // Re(conj a b)
__device__ __forceinline__ double crossc(cx<double> a, cx<double> b) { return a.x * b.y - a.y * b.x; } // Im(conj a b)

// One pass over the half spectrum accumulating, per block, the S FMT sums
//   sum_alpha Re[conj(dPhi_hat_alpha) dw_alpha^k/dR w_hat_k + conj(t_hat_alpha) dw_alpha^k/dR rho_hat_k]
// and for every ordered pair (i, j) the three screening-kernel sums
//   Re[conj(w_hat_i) K(k) drho_hat_j],  K = dC_ij/dlambda_i, dC_ij/dlambda_j, dC_ij/dR_c,
// each weighted 1 or 2 for the half spectrum (1 on the kx = 0 and Nyquist planes).
template <int MAXS>
__global__ __launch_bounds__(NTA) void k_adj_spec(Geo g, AdjSpecArgs a) {
    constexpr int NV = MAXS + 3 * MAXS * MAXS;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const Consts &c = *g.cs;
    const AdjConsts &ac = *a.ac;
    const int S = g.S;
    const cx<double> *Wh = reinterpret_cast<const cx<double> *>(a.wh);
    const cx<double> *Rh = reinterpret_cast<const cx<double> *>(a.rh);
    const cx<double> *Dh = reinterpret_cast<const cx<double> *>(a.dh);
    const cx<double> *Th = reinterpret_cast<const cx<double> *>(a.th);
    GRID_STRIDE(idx, g.NC) {
        const int kx = (int)(idx % g.Kx);
        const long long rest = idx / g.Kx;
        const int y = (int)(rest % g.ny);
        const int z = (int)(rest / g.ny);
        const double wt = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
        KInfo q;
        {
            const int my = signed_mode(y, c.ny), mz = signed_mode(z, c.nz);
            q.k[0] = kx * c.dk[0];
            q.k[1] = my * c.dk[1];
            q.k[2] = mz * c.dk[2];
            q.kmag = sqrt(q.k[0] * q.k[0] + q.k[1] * q.k[1] + q.k[2] * q.k[2]);
            q.nyq[0] = (c.nx % 2 == 0) && (2 * kx == c.nx);
            q.nyq[1] = (c.ny % 2 == 0) && (2 * y == c.ny);
            q.nyq[2] = (c.nz % 2 == 0) && (2 * z == c.nz);
            q.zero = kx == 0 && y == 0 && z == 0;
        }
        cx<double> D[DFT_NALPHA], T[DFT_NALPHA];
#pragma unroll
        for (int al = 0; al < DFT_NALPHA; ++al) {
            D[al] = Dh[(long long)al * g.NC + idx];
            T[al] = Th[(long long)al * g.NC + idx];
        }
        const double kd0 = k_comp(q, 0), kd1 = k_comp(q, 1), kd2 = k_comp(q, 2);
#pragma unroll
        for (int k = 0; k < MAXS; ++k) {
            if (k >= S) break;
            const double R = c.R[k];
            double j0, cy, g3;
            radial_fns(q.kmag, R, j0, cy, g3);
            const double dw0 = -q.kmag * q.kmag * R * g3;            // d/dR sin(kR)/(kR)
            const double dw1 = cy;                                     // d/dR sin(kR)/k
            const double dw2 = kFourPi * R * (j0 + cy);                // d/dR 4 pi R sin(kR)/k
            const double dw3 = kFourPi * R * R * j0;                   // d/dR w3 = w2
            const double xv1 = R * (j0 - g3);                          // w2/(4 pi R) - w3/(4 pi R^2)
            const double xv2 = kFourPi * R * R * j0;                   // w2
            const cx<double> Wk = Wh[(long long)k * g.NC + idx];
            const cx<double> Rk = Rh[(long long)k * g.NC + idx];
            double sum = dw0 * (dotc(D[0], Wk) + dotc(T[0], Rk)) + dw1 * (dotc(D[1], Wk) + dotc(T[1], Rk)) +
                         dw2 * (dotc(D[2], Wk) + dotc(T[2], Rk)) + dw3 * (dotc(D[3], Wk) + dotc(T[3], Rk));
            // vector weights: dw_V/dR = -i k_d X, Re[conj(a) (-i) b] = Im(conj(a) b)
            sum += xv1 * (kd0 * (crossc(D[4], Wk) + crossc(T[4], Rk)) + kd1 * (crossc(D[5], Wk) + crossc(T[5], Rk)) +
                          kd2 * (crossc(D[6], Wk) + crossc(T[6], Rk)));
            sum += xv2 * (kd0 * (crossc(D[7], Wk) + crossc(T[7], Rk)) + kd1 * (crossc(D[8], Wk) + crossc(T[8], Rk)) +
                          kd2 * (crossc(D[9], Wk) + crossc(T[9], Rk)));
            acc[k] += wt * sum;
        }
        if (c.es) {
#pragma unroll
            for (int i = 0; i < MAXS; ++i) {
                if (i >= S) break;
                const cx<double> Wi = Wh[(long long)i * g.NC + idx];
#pragma unroll
                for (int j = 0; j < MAXS; ++j) {
                    if (j >= S) break;
                    cx<double> dr = Rh[(long long)j * g.NC + idx];
                    if (q.zero) dr.x -= (double)c.N * c.rho_b[j];
                    const double base = wt * dotc(Wi, dr);
                    const int ij = i * DFT_MAX_SPECIES + j;
                    const double Rc = c.sc_R[ij];
                    double F1, F0, Fm1, j0c;
                    ball_moments(q.kmag, Rc, F1, F0, Fm1, j0c);
                    const double Kli = ac.li_c1[ij] * F1 + ac.li_c0[ij] * F0 + ac.li_cm1[ij] * Fm1;
                    const double Klj = ac.lj_c1[ij] * F1 + ac.lj_c0[ij] * F0 + ac.lj_cm1[ij] * Fm1;
                    const double Krc = kFourPi * j0c * Rc * (c.sc_c1[ij] * Rc * Rc + c.sc_c0[ij] * Rc + c.sc_cm1[ij]);
                    const int o = MAXS + 3 * (i * MAXS + j);
                    acc[o] += base * Kli;
                    acc[o + 1] += base * Klj;
                    acc[o + 2] += base * Krc;
                }
            }
        }
    }
    block_partials<NV>(acc, a.part + (long long)blockIdx.x * NV);
}

// ---------------------------------------------------------------- launchers
static unsigned nblk(long long n) { return (unsigned)std::min<long long>((n + NTA - 1) / NTA, 2048); }

void adj_init(long long n, const double *G, const double *g, double *w, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_init, dim3(nblk(n)), dim3(NTA), 0, s, n, G, g, w);
    check_launch_a("adj_init");
}

int adj_r0(long long n, const double *G, const double *Hw, double *r, double *p, double *part, hipStream_t s) {
    const unsigned nb = nblk(n);
    hipLaunchKernelGGL(k_adj_r0, dim3(nb), dim3(NTA), 0, s, n, G, Hw, r, p, part);
    check_launch_a("adj_r0");
    return (int)nb;
}

int adj_q(long long n, const double *G, const double *p, const double *Hp, double *q, double *part, hipStream_t s) {
    const unsigned nb = nblk(n);
    hipLaunchKernelGGL(k_adj_q, dim3(nb), dim3(NTA), 0, s, n, G, p, Hp, q, part);
    check_launch_a("adj_q");
    return (int)nb;
}

int adj_step(long long n, double alpha, const double *G, const double *p, const double *q, double *w, double *r,
             double *part, hipStream_t s) {
    const unsigned nb = nblk(n);
    hipLaunchKernelGGL(k_adj_step, dim3(nb), dim3(NTA), 0, s, n, alpha, G, p, q, w, r, part);
    check_launch_a("adj_step");
    return (int)nb;
}

void adj_dir(long long n, double beta, const double *G, const double *r, double *p, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_dir, dim3(nblk(n)), dim3(NTA), 0, s, n, beta, G, r, p);
    check_launch_a("adj_dir");
}

int adj_fieldsum(long long N, int S, const double *f, double *part, hipStream_t s) {
    const unsigned nb = nblk(N);
    hipLaunchKernelGGL(k_adj_fieldsum, dim3(nb, S), dim3(NTA), 0, s, N, f, part);
    check_launch_a("adj_fieldsum");
    return (int)nb;
}

void adj_neg(long long n, const double *w, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_neg, dim3(nblk(n)), dim3(NTA), 0, s, n, w, out);
    check_launch_a("adj_neg");
}

void newton_rhs(long long n, const double *G, const double *rho, double *g, hipStream_t s) {
    hipLaunchKernelGGL(k_newton_rhs, dim3(nblk(n)), dim3(NTA), 0, s, n, G, rho, g);
    check_launch_a("newton_rhs");
}

int newton_bound(long long n, const double *rho, const double *d, double *part, hipStream_t s) {
    const int nb = nblk(n);
    hipLaunchKernelGGL(k_newton_bound, dim3(nb), dim3(NTA), 0, s, n, rho, d, part);
    check_launch_a("newton_bound");
    return nb;
}

void axpy(long long n, const double *x, double a, const double *d, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(NTA), 0, s, n, x, a, d, out);
    check_launch_a("axpy");
}

void adj_reduce(const double *part, int nparts, int nv, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(NTA), 0, s, part, nparts, nv, out);
    check_launch_a("adj_reduce");
}

int adj_spec(const Geo &g, const AdjSpecArgs &a, hipStream_t s) {
    if (g.S > 4) throw std::runtime_error("adjoint gradients support at most 4 species");
    const unsigned nb = nblk(g.NC);
    hipLaunchKernelGGL((k_adj_spec<4>), dim3(nb), dim3(NTA), 0, s, g, a);
    check_launch_a("adj_spec");
    return (int)nb;
}

}  // namespace dft
