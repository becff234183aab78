// Pass kernels of one residual evaluation G(rho) for gfx950.
//
// A residual evaluation is nine streaming passes over HBM (one per axis and direction),
// with the method's pointwise and spectral work fused into them:
//   X1  x: real rows -> half spectra (forward; forms the line-search trial point)
//   Y1  y: forward
//   Z1  z: forward, spectral products with the weight transforms (eqs. nDef, conv,
//          Appendix B), inverse z -> ten weighted-density spectra
//   Y2  y: inverse
//   X2  x: inverse to real n_alpha, pointwise dPhi/dn_alpha (eq. Phi), forward again
//   Y3  y: forward
//   Z2  z: forward, back-convolution with conj(w_hat) (eq. muHS), bulk-fluid screening
//          (eq. muESexpansion) and the Poisson solve (eq. potentialSolution), inverse z
//   Y4  y: inverse
//   X3  x: inverse to real E_k, Euler-Lagrange update (eq. rhoEquation) and residual sums
// Each pass reads and writes every field once; the 1/N of the inverse transform is
// applied in the z passes.  Transforms are LDS-staged mixed-radix Stockham FFTs over
// tiles of pencils whose global accesses are contiguous along x.
#include "dft_kernels.h"
#include "pass_util.h"

#include <cmath>
#include <cstdio>
#include <stdexcept>
#include <type_traits>

namespace dft {

constexpr int NT = 256;

template <typename T> struct Cfg;
template <> struct Cfg<double> {
    static constexpr int XE = 8, X2E = 4, YE = 8, ZE = 4, WMAX = 8;
};
template <> struct Cfg<float> {
    static constexpr int XE = 16, X2E = 4, YE = 16, ZE = 4, WMAX = 16;
};

template <bool MAX>
__device__ __forceinline__ void block_reduce(double v, int fl, double *dst, int *fdst) {
    block_reduce_nt<MAX, NT>(v, fl, dst, fdst);
}

// --------------------------------------------------------------------- x passes
// Two real rows (r0, r1) travel as the real and imaginary parts of one complex row:
// a forward FFT of c = a + i b gives A_k = (C_k + conj C_{L-k}) / 2 and
// B_k = (C_k - conj C_{L-k}) / (2i); the inverse rebuilds C from the Hermitian halves.

template <typename T>
__device__ __forceinline__ void x_store_halves(const cx<T> *tile, int L, int Kx, int Pact, long long pair0,
                                               long long rows, cx<T> *out) {
    for (int j = threadIdx.x; j < Pact * Kx; j += NT) {
        const int pl = j / Kx, k = j - pl * Kx;
        const cx<T> ck = tile[pl * L + k];
        const cx<T> cm = tile[pl * L + (k == 0 ? 0 : L - k)];
        const long long r0 = 2 * (pair0 + pl);
        out[r0 * Kx + k] = mk<T>(T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y - cm.y));
        if (r0 + 1 < rows) out[(r0 + 1) * Kx + k] = mk<T>(T(0.5) * (ck.y + cm.y), T(-0.5) * (ck.x - cm.x));
    }
}

template <typename T>
__device__ __forceinline__ cx<T> x_half_at(const cx<T> *row, int e, int L, int Kx) {
    cx<T> v;
    if (e < Kx) {
        v = row[e];
        if (e == 0 || 2 * e == L) v.y = T(0);
    } else {
        v = conjg(row[L - e]);
    }
    return v;
}

template <typename T>
__device__ __forceinline__ void x_load_halves(cx<T> *tile, int L, int Kx, int Pact, long long pair0, long long rows,
                                              const cx<T> *in) {
    for (int j = threadIdx.x; j < Pact * L; j += NT) {
        const int pl = j / L, e = j - pl * L;
        const long long r0 = 2 * (pair0 + pl);
        const cx<T> A = x_half_at(in + r0 * Kx, e, L, Kx);
        cx<T> B = mk<T>(T(0), T(0));
        if (r0 + 1 < rows) B = x_half_at(in + (r0 + 1) * Kx, e, L, Kx);
        tile[pl * L + e] = mk<T>(A.x - B.y, A.y + B.x);
    }
}

template <typename T, int MAXE>
__global__ __launch_bounds__(NT) void k_x_forward(Geo g_in, XFwdArgs a, int P) {
    const int prob_ = (int)blockIdx.z / (1);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    resolve_roles(a);
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const int f = blockIdx.y;
    const int L = g.nx, Kx = g.Kx;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * P;
    const int Pact = (int)min((long long)P, npairs - pair0);
    const long long foff = (long long)f * g.N;
    const double alpha = (a.mode == XF_TRIAL) ? *a.alpha : 0.0;
    for (int j = threadIdx.x; j < Pact * L; j += NT) {
        const int pl = j / L, e = j - pl * L;
        const long long r0 = 2 * (pair0 + pl);
        double v[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long r = r0 + h;
            if (r >= rows) break;
            const long long idx = foff + r * L + e;
            double x;
            if (a.mode == XF_TRIAL) {
                const double r0v = a.src[idx];
                x = fma(alpha, a.g0[idx] - r0v, r0v);
                if (a.rho_t) a.rho_t[idx] = x;
            } else {
                x = a.src[idx];
            }
            if (a.ref) x -= a.ref[idx];
            v[h] = x;
        }
        tile[j] = mk<T>(T(v[0]), T(v[1]));
    }
    __syncthreads();
    fft_tile<T, -1, NT, MAXE>(tile, g.px, Pact, 1, L, true, twp<T>(g, 0));
    x_store_halves<T>(tile, L, Kx, Pact, pair0, rows, reinterpret_cast<cx<T> *>(a.spec) + (long long)f * g.NC);
}

// --------------------------------------------------------------------- y passes
template <typename T, int MAXE>
__global__ __launch_bounds__(NT) void k_y(Geo g_in, YArgs a, int W) {
    const int prob_ = (int)blockIdx.z / (a.nfield);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const bool zax = a.axis == 2;
    const int L = zax ? g.nz : g.ny, Kx = g.Kx;
    int bx, o;
    xcd_block(bx, o);
    const int kx0 = bx * W;
    const int Wact = min(W, Kx - kx0);
    const int f = (int)blockIdx.z % a.nfield;
    // y: rows of one z plane (stride Kx); z: one y line through every plane (stride ny Kx)
    const long long rs = zax ? (long long)g.ny * Kx : (long long)Kx;
    const long long ob = zax ? (long long)o * Kx : (long long)o * g.ny * Kx;
    cx<T> *base = reinterpret_cast<cx<T> *>(a.spec) + (long long)f * g.NC + ob + kx0;
    for (int j = threadIdx.x; j < Wact * L; j += NT) {
        const int e = j / Wact, p = j - e * Wact;
        tile[j] = base[(long long)e * rs + p];
    }
    __syncthreads();
    fft_tile_dir<T, NT, MAXE>(a.dir, tile, zax ? g.pz : g.py, Wact, Wact, 1, false, twp<T>(g, zax ? 2 : 1));
    for (int j = threadIdx.x; j < Wact * L; j += NT) {
        const int e = j / Wact, p = j - e * Wact;
        base[(long long)e * rs + p] = tile[j];
    }
}

// --------------------------------------------------------------------- z passes
template <typename T>
__device__ __forceinline__ void z_load(cx<T> *tile, const cx<T> *src, int Wact, int L, long long rowstride) {
    for (int j = threadIdx.x; j < Wact * L; j += NT) {
        const int e = j / Wact, p = j - e * Wact;
        tile[j] = src[(long long)e * rowstride + p];
    }
}
template <typename T>
__device__ __forceinline__ void z_store(const cx<T> *tile, cx<T> *dst, int Wact, int L, long long rowstride) {
    for (int j = threadIdx.x; j < Wact * L; j += NT) {
        const int e = j / Wact, p = j - e * Wact;
        dst[(long long)e * rowstride + p] = tile[j];
    }
}

// Z1: forward z transform of every species, then
//   (a) the five weighted sums of Appendix B spectra that give the ten n_alpha spectra
//       (the vector spectra are -i k times a w3 sum), inverse z -> specB;
//   (b) with electrostatics, per species i the linear electrostatic part of the exponent
//       sum_j [C_ij(k) - z_i z_j 4 pi l_B / D(k)] (rho_hat_j - N rho_b_j delta_k0)
//       (eqs. muESexpansion, potentialSolution), written unnormalized over rho_hat in specA.
// Spectral factors are evaluated in the transform precision T.
template <typename T, int MAXE, int MAXS>
__global__ __launch_bounds__(NT) void k_z1(Geo g_in, Z1Args a, int W) {
    const int prob_ = (int)blockIdx.z / (1);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const Consts &c = *g.cs;
    const int L = g.nz, Kx = g.Kx, S = g.S;
    int bx, y;
    xcd_block(bx, y);
    const int kx0 = bx * W;
    const int Wact = min(W, Kx - kx0);
    const long long rs = (long long)g.ny * Kx;
    const long long off = (long long)y * Kx + kx0;
    const cx<T> *tw = twp<T>(g, 2);
    const bool es = c.es && !a.n3only;
    T kmag[MAXE], invD[MAXE];
    bool kzero[MAXE];
#pragma unroll
    for (int it = 0; it < MAXE; ++it) {
        const int j = threadIdx.x + it * NT;
        kmag[it] = T(0);
        invD[it] = T(0);
        kzero[it] = false;
        if (j < Wact * L) {
            const int e = j / Wact, p = j - e * Wact;
            const KInfo q = kinfo(c, kx0 + p, y, e);
            kmag[it] = T(q.kmag);
            kzero[it] = q.zero;
            if (es && !q.zero) {
                const T kd[3] = {T(q.k[0]), T(q.k[1]), T(q.k[2])};
                invD[it] = T(c.four_pi_lB) / poisson_denominator<T>(kd, c.h);
            }
        }
    }
    T acc[5][MAXE][2];
    T esa[MAXS][MAXE][2];
#pragma unroll
    for (int it = 0; it < MAXE; ++it) {
#pragma unroll
        for (int m = 0; m < 5; ++m) acc[m][it][0] = acc[m][it][1] = T(0);
#pragma unroll
        for (int m = 0; m < MAXS; ++m) esa[m][it][0] = esa[m][it][1] = T(0);
    }
    for (int jsp = 0; jsp < S; ++jsp) {
        const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specA) + (long long)jsp * g.NC + off;
        z_load(tile, src, Wact, L, rs);
        __syncthreads();
        fft_tile<T, -1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
        const T Rj = T(c.R[jsp]), a0 = T(c.i4piR2[jsp]), a1 = T(c.i4piR[jsp]);
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Wact * L) {
                const cx<T> v = tile[j];
                T w2, w3;
                weight_w2_w3<T>(kmag[it], Rj, w2, w3);
                const T m0 = w2 * a0, m1 = w2 * a1, m4 = w3 * a1;
                acc[0][it][0] += v.x * m0; acc[0][it][1] += v.y * m0;
                acc[1][it][0] += v.x * m1; acc[1][it][1] += v.y * m1;
                acc[2][it][0] += v.x * w2; acc[2][it][1] += v.y * w2;
                acc[3][it][0] += v.x * w3; acc[3][it][1] += v.y * w3;
                acc[4][it][0] += v.x * m4; acc[4][it][1] += v.y * m4;
                if (es) {
                    T vx = v.x;
                    if (kzero[it] && !a.diff) vx -= T((double)c.N * c.rho_b[jsp]);
#pragma unroll
                    for (int i = 0; i < MAXS; ++i) {
                        if (i < S) {
                            const int ij = i * DFT_MAX_SPECIES + jsp;
                            const T C = screening_hat<T>(kmag[it], T(c.sc_R[ij]), T(c.sc_c1[ij]), T(c.sc_c0[ij]),
                                                         T(c.sc_cm1[ij]));
                            const T P = invD[it] * T(c.z[i] * c.z[jsp]);
                            esa[i][it][0] += C * vx - P * v.x;
                            esa[i][it][1] += (C - P) * v.y;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (es) {
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            if (i >= S) break;
            cx<T> *dst = reinterpret_cast<cx<T> *>(a.specA) + (long long)i * g.NC + off;
#pragma unroll
            for (int it = 0; it < MAXE; ++it) {
                const int j = threadIdx.x + it * NT;
                if (j < Wact * L) {
                    const int e = j / Wact, p = j - e * Wact;
                    dst[(long long)e * rs + p] = mk<T>(esa[i][it][0], esa[i][it][1]);
                }
            }
        }
    }
    const int nout = a.n3only ? 1 : DFT_NALPHA;
    const T invN = T(c.invN);
    for (int o = 0; o < nout; ++o) {
        const int alpha = a.n3only ? 3 : o;
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Wact * L) {
                const int e = j / Wact, p = j - e * Wact;
                // select the source sum with compile-time register indices
                T sx = T(0), sy = T(0);
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    const bool pick = (alpha < 4) ? (m == alpha) : (m == (alpha < 7 ? 4 : 3));
                    if (pick) { sx = acc[m][it][0]; sy = acc[m][it][1]; }
                }
                T re = sx, im = sy;
                if (alpha >= 4) {
                    const int d = (alpha - 4) % 3;
                    const KInfo q = kinfo(c, kx0 + p, y, e);
                    const T kd = T(k_comp(q, d));
                    // -i k_d s
                    re = kd * sy;
                    im = -kd * sx;
                }
                tile[j] = mk<T>(re * invN, im * invN);
            }
        }
        __syncthreads();
        fft_tile<T, 1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
        z_store(tile, reinterpret_cast<cx<T> *>(a.specB) + (long long)o * g.NC + off, Wact, L, rs);
        __syncthreads();
    }
}

// Z2: forward z transform of the ten dPhi/dn spectra, back-convolution with conj(w_hat)
// (eq. muHS; the vector parts enter as +i k_d times a w3 weight), plus the electrostatic
// spectra Z1 left in specA, times 1/N, inverse z -> specA.  Z2_POISSON instead forms the
// potential of weighted source spectra.
template <typename T, int MAXE>
__global__ __launch_bounds__(NT) void k_z2(Geo g_in, Z2Args a, int W) {
    const int prob_ = (int)blockIdx.z / (1);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const Consts &c = *g.cs;
    const int L = g.nz, Kx = g.Kx;
    int bx, y;
    xcd_block(bx, y);
    const int kx0 = bx * W;
    const int Wact = min(W, Kx - kx0);
    const long long rs = (long long)g.ny * Kx;
    const long long off = (long long)y * Kx + kx0;
    const cx<T> *tw = twp<T>(g, 2);
    const int S = g.S;

    if (a.mode == Z2_BALL) {
        // ball average of every source field at one radius: specA[i] x B(|k| radius) / N -> specB[i]
        for (int i = 0; i < a.nsrc; ++i) {
            const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specA) + (long long)i * g.NC + off;
            z_load(tile, src, Wact, L, rs);
            __syncthreads();
            fft_tile<T, -1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
#pragma unroll
            for (int it = 0; it < MAXE; ++it) {
                const int j = threadIdx.x + it * NT;
                if (j < Wact * L) {
                    const int e = j / Wact, p = j - e * Wact;
                    const KInfo q = kinfo(c, kx0 + p, y, e);
                    const double m = ball_mean<double>(q.kmag, a.radius) * c.invN;
                    tile[j] = mk<T>(T((double)tile[j].x * m), T((double)tile[j].y * m));
                }
            }
            __syncthreads();
            fft_tile<T, 1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
            z_store(tile, reinterpret_cast<cx<T> *>(a.specB) + (long long)i * g.NC + off, Wact, L, rs);
            __syncthreads();
        }
        return;
    }
    if (a.mode == Z2_POISSON) {
        // phi_hat = 4 pi l_B (sum_j w_j src_j) / D(k), zero mode 0; x invN; output in specA[0].
        double acc[MAXE][2];
#pragma unroll
        for (int it = 0; it < MAXE; ++it) acc[it][0] = acc[it][1] = 0.0;
        for (int i = 0; i < a.nsrc; ++i) {
            const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specA) + (long long)i * g.NC + off;
            z_load(tile, src, Wact, L, rs);
            __syncthreads();
            fft_tile<T, -1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
#pragma unroll
            for (int it = 0; it < MAXE; ++it) {
                const int j = threadIdx.x + it * NT;
                if (j < Wact * L) {
                    acc[it][0] += a.wsrc[i] * (double)tile[j].x;
                    acc[it][1] += a.wsrc[i] * (double)tile[j].y;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Wact * L) {
                const int e = j / Wact, p = j - e * Wact;
                const KInfo q = kinfo(c, kx0 + p, y, e);
                double m = 0.0;
                if (!q.zero) m = c.four_pi_lB / poisson_denominator<double>(q.k, c.h) * c.invN;
                tile[j] = mk<T>(T(acc[it][0] * m), T(acc[it][1] * m));
            }
        }
        __syncthreads();
        fft_tile<T, 1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
        z_store(tile, reinterpret_cast<cx<T> *>(a.specA) + off, Wact, L, rs);
        return;
    }

    // six sums of the derivative spectra: u0..u3 and v1 = sum_d i k_d dPhi_V1,d, v2 likewise
    T u[6][MAXE][2];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int it = 0; it < MAXE; ++it) u[m][it][0] = u[m][it][1] = T(0);
    for (int al = 0; al < DFT_NALPHA; ++al) {
        const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specB) + (long long)al * g.NC + off;
        z_load(tile, src, Wact, L, rs);
        __syncthreads();
        fft_tile<T, -1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Wact * L) {
                T vx = tile[j].x, vy = tile[j].y;
                if (al >= 4) {
                    const int e = j / Wact, p = j - e * Wact;
                    const int d = (al - 4) % 3;
                    const KInfo q = kinfo(c, kx0 + p, y, e);
                    const T kd = T(k_comp(q, d));
                    // + i k_d v
                    const T tx = -kd * vy;
                    vy = kd * vx;
                    vx = tx;
                }
                const int m = al < 4 ? al : (al < 7 ? 4 : 5);
#pragma unroll
                for (int mm = 0; mm < 6; ++mm)
                    if (mm == m) { u[mm][it][0] += vx; u[mm][it][1] += vy; }
            }
        }
        __syncthreads();
    }
    const T invN = T(c.invN);
    for (int i = 0; i < S; ++i) {
        const T Ri = T(c.R[i]), a0 = T(c.i4piR2[i]), a1 = T(c.i4piR[i]);
        const cx<T> *esrc = reinterpret_cast<const cx<T> *>(a.specA) + (long long)i * g.NC + off;
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Wact * L) {
                const int e = j / Wact, p = j - e * Wact;
                const KInfo q = kinfo(c, kx0 + p, y, e);
                T w2, w3;
                weight_w2_w3<T>(T(q.kmag), Ri, w2, w3);
                const T s2x = u[0][it][0] * a0 + u[1][it][0] * a1 + u[2][it][0];
                const T s2y = u[0][it][1] * a0 + u[1][it][1] * a1 + u[2][it][1];
                const T s3x = u[3][it][0] + u[4][it][0] * a1 + u[5][it][0];
                const T s3y = u[3][it][1] + u[4][it][1] * a1 + u[5][it][1];
                T ex = -(s2x * w2 + s3x * w3);
                T ey = -(s2y * w2 + s3y * w3);
                if (c.es) {
                    const cx<T> ev = esrc[(long long)e * rs + p];
                    ex += ev.x;
                    ey += ev.y;
                }
                tile[j] = mk<T>(ex * invN, ey * invN);
            }
        }
        __syncthreads();
        fft_tile<T, 1, NT, MAXE>(tile, g.pz, Wact, Wact, 1, false, tw);
        z_store(tile, reinterpret_cast<cx<T> *>(a.specA) + (long long)i * g.NC + off, Wact, L, rs);
        __syncthreads();
    }
}

// --------------------------------------------------------------------- X2: pointwise FMT
template <typename T, int MAXE>
__global__ __launch_bounds__(NT) void k_x2(Geo g_in, X2Args a, int P) {
    const int prob_ = (int)blockIdx.z / (1);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const int L = g.nx, Kx = g.Kx;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * P;
    const int Pact = (int)min((long long)P, npairs - pair0);
    const cx<T> *tw = twp<T>(g, 0);
    const bool n3only = a.mode == X2_N3_ONLY;
    const int nf = n3only ? 1 : DFT_NALPHA;
    double nv[DFT_NALPHA][MAXE][2];
    for (int f = 0; f < nf; ++f) {
        x_load_halves<T>(tile, L, Kx, Pact, pair0, rows, reinterpret_cast<const cx<T> *>(a.specB) + (long long)f * g.NC);
        __syncthreads();
        fft_tile<T, 1, NT, MAXE>(tile, g.px, Pact, 1, L, true, tw);
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Pact * L) {
                const double vx = (double)tile[j].x, vy = (double)tile[j].y;
#pragma unroll
                for (int ff = 0; ff < DFT_NALPHA; ++ff)
                    if (ff == f) { nv[ff][it][0] = vx; nv[ff][it][1] = vy; }
            }
        }
        __syncthreads();
    }
    double mloc = -INFINITY;
    int flag = 0;
#pragma unroll
    for (int it = 0; it < MAXE; ++it) {
        const int j = threadIdx.x + it * NT;
        if (j >= Pact * L) continue;
        const int pl = j / L, e = j - pl * L;
        const long long r0 = 2 * (pair0 + pl);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long r = r0 + h;
            if (r >= rows) {
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) nv[f][it][h] = 0.0;
                continue;
            }
            const long long idx = r * L + e;
            if (n3only) {
                double n3 = nv[0][it][h];
                if (a.nref) n3 += (double)a.nref[3 * g.N + idx];
                if (!isfinite(n3)) flag |= 5;   // 1: evaluation non-finite, 4: n3 non-finite
                mloc = fmax(mloc, n3);
                continue;
            }
            double n[DFT_NALPHA], d[DFT_NALPHA];
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) n[f] = nv[f][it][h];
            bool clamped = false;
            if (a.nref) {
                double nr[DFT_NALPHA], dr[DFT_NALPHA];
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) {
                    nr[f] = (double)a.nref[f * g.N + idx];
                    n[f] += nr[f];
                }
                bool c2;
                fmt_dphi_sel<double>(a.hs, n, d, clamped);
                fmt_dphi_sel<double>(a.hs, nr, dr, c2);
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) d[f] -= dr[f];
            } else {
                fmt_dphi_sel<double>(a.hs, n, d, clamped);
            }
            if (clamped) flag |= 2;
            if (!isfinite(n[3])) flag |= 5;
            if (!isfinite(d[0]) || !isfinite(d[3])) flag |= 1;
            mloc = fmax(mloc, n[3]);
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) {
                if (a.nref_out) a.nref_out[f * g.N + idx] = (float)n[f];
                if (a.n_out) a.n_out[f * g.N + idx] = n[f];
                if (a.dphi_out) a.dphi_out[f * g.N + idx] = d[f];
                nv[f][it][h] = d[f];
            }
        }
    }
    if (flag & 4) mloc = INFINITY;   // the n3 bound needs finite n3 only
    block_reduce<true>(mloc, flag, a.red.mpart + blockIdx.x, a.red.mflag + blockIdx.x);
    if (n3only) return;
    __syncthreads();
    for (int f = 0; f < DFT_NALPHA; ++f) {
#pragma unroll
        for (int it = 0; it < MAXE; ++it) {
            const int j = threadIdx.x + it * NT;
            if (j < Pact * L) {
                double vx = 0.0, vy = 0.0;
#pragma unroll
                for (int ff = 0; ff < DFT_NALPHA; ++ff)
                    if (ff == f) { vx = nv[ff][it][0]; vy = nv[ff][it][1]; }
                tile[j] = mk<T>(T(vx), T(vy));
            }
        }
        __syncthreads();
        fft_tile<T, -1, NT, MAXE>(tile, g.px, Pact, 1, L, true, tw);
        x_store_halves<T>(tile, L, Kx, Pact, pair0, rows, reinterpret_cast<cx<T> *>(a.specB) + (long long)f * g.NC);
        __syncthreads();
    }
}

// Batched variant: all ten fields of PB row pairs sit in LDS as 10*PB pencils, so each
// direction is one FFT over the batch (one barrier pair per stage for all fields) and
// the pointwise work reads and writes LDS instead of holding the fields in registers.
template <typename T, int NTB, int MAXE>
__global__ __launch_bounds__(NTB) void k_x2b(Geo g_in, X2Args a, int PB) {
    const int prob_ = (int)blockIdx.z / (1);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const int L = g.nx, Kx = g.Kx;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * PB;
    const int Pact = (int)min((long long)PB, npairs - pair0);
    const cx<T> *tw = twp<T>(g, 0);
    const bool n3only = a.mode == X2_N3_ONLY;
    const int nf = n3only ? 1 : DFT_NALPHA;
    const int span = Pact * L;          // elements of one field in the tile
    const int P = nf * Pact;            // pencils in the batch
    for (int j = threadIdx.x; j < P * L; j += NTB) {
        const int f = j / span;
        const int jj = j - f * span;
        const int pl = jj / L, e = jj - pl * L;
        const long long r0 = 2 * (pair0 + pl);
        const cx<T> *in = reinterpret_cast<const cx<T> *>(a.specB) + (long long)f * g.NC;
        const cx<T> A = x_half_at(in + r0 * Kx, e, L, Kx);
        cx<T> B = mk<T>(T(0), T(0));
        if (r0 + 1 < rows) B = x_half_at(in + (r0 + 1) * Kx, e, L, Kx);
        tile[j] = mk<T>(A.x - B.y, A.y + B.x);
    }
    __syncthreads();
    fft_tile<T, 1, NTB, MAXE>(tile, g.px, P, 1, L, true, tw);
    double mloc = -INFINITY;
    int flag = 0;
    for (int jj = threadIdx.x; jj < span; jj += NTB) {
        const int pl = jj / L, e = jj - pl * L;
        const long long r0 = 2 * (pair0 + pl);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long r = r0 + h;
            if (r >= rows) break;
            const long long idx = r * L + e;
            if (n3only) {
                double n3 = h == 0 ? (double)tile[jj].x : (double)tile[jj].y;
                if (a.nref) n3 += (double)a.nref[3 * g.N + idx];
                if (!isfinite(n3)) flag |= 5;   // 1: evaluation non-finite, 4: n3 non-finite
                mloc = fmax(mloc, n3);
                continue;
            }
            double n[DFT_NALPHA], d[DFT_NALPHA];
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) {
                const cx<T> v = tile[f * span + jj];
                n[f] = h == 0 ? (double)v.x : (double)v.y;
            }
            bool clamped = false;
            if (a.mode == X2_HESS) {
                // t = Phi''(n*) n by forward-mode differentiation of dPhi/dn at n*
                Dual nd[DFT_NALPHA], dd[DFT_NALPHA];
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) nd[f] = Dual{a.nstar[f * g.N + idx], n[f]};
                fmt_dphi_sel<Dual>(a.hs, nd, dd, clamped);
                bool bad = false;
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) {
                    d[f] = dd[f].d;
                    bad |= !isfinite(d[f]);
                    if (a.t_out) a.t_out[f * g.N + idx] = d[f];
                    if (h == 0) tile[f * span + jj].x = T(d[f]);
                    else tile[f * span + jj].y = T(d[f]);
                }
                if (bad) flag |= 1;
                continue;
            }
            if (a.nref) {
                double nr[DFT_NALPHA], dr[DFT_NALPHA];
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) {
                    nr[f] = (double)a.nref[f * g.N + idx];
                    n[f] += nr[f];
                }
                bool c2;
                fmt_dphi_sel<double>(a.hs, n, d, clamped);
                fmt_dphi_sel<double>(a.hs, nr, dr, c2);
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) d[f] -= dr[f];
            } else {
                fmt_dphi_sel<double>(a.hs, n, d, clamped);
            }
            if (clamped) flag |= 2;
            if (!isfinite(n[3])) flag |= 5;
            if (!isfinite(d[0]) || !isfinite(d[3])) flag |= 1;
            mloc = fmax(mloc, n[3]);
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) {
                if (a.nref_out) a.nref_out[f * g.N + idx] = (float)n[f];
                if (a.n_out) a.n_out[f * g.N + idx] = n[f];
                if (a.dphi_out) a.dphi_out[f * g.N + idx] = d[f];
                if (h == 0) tile[f * span + jj].x = T(d[f]);
                else tile[f * span + jj].y = T(d[f]);
            }
        }
        if (!n3only && r0 + 1 >= rows) {
            // the missing partner row transforms as zero
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) tile[f * span + jj].y = T(0);
        }
    }
    if (flag & 4) mloc = INFINITY;   // the n3 bound needs finite n3 only
    block_reduce_nt<true, NTB>(mloc, flag, a.red.mpart + blockIdx.x, a.red.mflag + blockIdx.x);
    if (n3only) return;
    __syncthreads();
    fft_tile<T, -1, NTB, MAXE>(tile, g.px, P, 1, L, true, tw);
    for (int j = threadIdx.x; j < nf * Pact * Kx; j += NTB) {
        const int f = j / (Pact * Kx);
        const int jj = j - f * (Pact * Kx);
        const int pl = jj / Kx, k = jj - pl * Kx;
        const cx<T> *tf = tile + f * span;
        const cx<T> ck = tf[pl * L + k];
        const cx<T> cm = tf[pl * L + (k == 0 ? 0 : L - k)];
        const long long r0 = 2 * (pair0 + pl);
        cx<T> *out = reinterpret_cast<cx<T> *>(a.specB) + (long long)f * g.NC;
        out[r0 * Kx + k] = mk<T>(T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y - cm.y));
        if (r0 + 1 < rows) out[(r0 + 1) * Kx + k] = mk<T>(T(0.5) * (ck.y + cm.y), T(-0.5) * (ck.x - cm.x));
    }
}

// --------------------------------------------------------------------- X3: Euler-Lagrange update
template <typename T, int MAXE>
__global__ __launch_bounds__(NT) void k_x3(Geo g_in, X3Args a, int P) {
    const int prob_ = (int)blockIdx.z / (1);
    if (prob_ > 0) {
        const long long off_ = (long long)prob_ * g_in.pstride;
        g_in = shift(g_in, off_);
        a = shift(a, off_);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    resolve_roles(a);
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);
    const Consts &c = *g.cs;
    const int i = blockIdx.y;
    const int L = g.nx, Kx = g.Kx;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * P;
    const int Pact = (int)min((long long)P, npairs - pair0);
    x_load_halves<T>(tile, L, Kx, Pact, pair0, rows, reinterpret_cast<const cx<T> *>(a.specA) + (long long)i * g.NC);
    __syncthreads();
    fft_tile<T, 1, NT, MAXE>(tile, g.px, Pact, 1, L, true, twp<T>(g, 0));
    double acc = 0.0;
    int flag = 0;
    const double rb = c.rho_b[i], irb = c.inv_rho_b[i];
    for (int j = threadIdx.x; j < Pact * L; j += NT) {
        const int pl = j / L, e = j - pl * L;
        const long long r0 = 2 * (pair0 + pl);
        const cx<T> v = tile[j];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long r = r0 + h;
            if (r >= rows) break;
            const double E = h == 0 ? (double)v.x : (double)v.y;
            const long long idx = (long long)i * g.N + r * L + e;
            if (a.raw) {
                double o = E;
                if (a.addend) o += a.addend[r * L + e];
                a.raw_out[idx] = o;
                continue;
            }
            const double b = a.base[idx];
            const bool fluid = b > -INFINITY;
            const double G = fluid ? rb * exp(b + E) : 0.0;
            if (a.g_out) a.g_out[idx] = G;
            if (a.e_out) a.e_out[idx] = a.e_phi ? E - c.z[i] * a.e_phi[r * L + e] : E;
            if (a.lp_out) a.lp_out[idx] = fluid ? b + E : -INFINITY;
            if (fluid) {
                const double dlt = (a.rho_t[idx] - G) * irb;
                acc += dlt * dlt;
                if (!isfinite(G)) flag |= 1;
            }
        }
    }
    if (a.raw) return;
    block_reduce<false>(acc, flag, a.red.fpart + (long long)blockIdx.y * gridDim.x + blockIdx.x,
                        a.red.fflag + (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// --------------------------------------------------------------------- launch geometry
static void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T, int MAXE>
static int x_pairs(const Geo &g) {
    int P = (NT * MAXE) / g.nx;
    if (P < 1) throw std::runtime_error("x pass: row longer than one tile");
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    if (P > npairs) P = (int)npairs;
    return P;
}

template <typename T, int MAXE>
static int yz_width(int L, int Kx) {
    int W = (NT * MAXE) / L;
    if (W > Cfg<T>::WMAX) W = Cfg<T>::WMAX;
    if (W > Kx) W = Kx;
    if (W < 1) throw std::runtime_error("y/z pass: pencil longer than one tile");
    return W;
}

static long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

template <typename T>
void launch_x_forward(const Geo &g, const XFwdArgs &a, hipStream_t s) {
    if (launch_x1_ct<T>(g, a, s)) return;
    constexpr int E = Cfg<T>::XE;
    const int P = x_pairs<T, E>(g);
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    dim3 grid((unsigned)ceil_div(npairs, P), (unsigned)a.nfield, (unsigned)g.nprob);
    const size_t sh = (size_t)P * g.nx * sizeof(cx<T>);
    hipLaunchKernelGGL((k_x_forward<T, E>), grid, dim3(NT), sh, s, g, a, P);
    check_launch("x_forward");
}

template <typename T>
void launch_y(const Geo &g, const YArgs &a, hipStream_t s) {
    const bool zax = a.axis == 2;
    const int L = zax ? g.nz : g.ny;
    if (L == 1) return;   // a length-1 transform is the identity
    if (launch_y_ct<T>(g, a, s)) return;
    if (a.vec) throw std::runtime_error("y: compact vector layout without a compiled-length kernel");
    constexpr int E = Cfg<T>::YE;
    const int W = yz_width<T, E>(L, g.Kx);
    dim3 grid((unsigned)ceil_div(g.Kx, W), (unsigned)(zax ? g.ny : g.nz), (unsigned)(a.nfield * g.nprob));
    const size_t sh = (size_t)W * L * sizeof(cx<T>);
    hipLaunchKernelGGL((k_y<T, E>), grid, dim3(NT), sh, s, g, a, W);
    check_launch("y");
}

template <typename T>
void launch_z1(const Geo &g, const Z1Args &a, hipStream_t s) {
    if (launch_z1_ct<T>(g, a, g.es && !a.n3only, s)) return;
    if (g.compact) throw std::runtime_error("z1: compact vector layout without a compiled-length kernel");
    constexpr int E = Cfg<T>::ZE;
    const int W = yz_width<T, E>(g.nz, g.Kx);
    dim3 grid((unsigned)ceil_div(g.Kx, W), (unsigned)g.ny, (unsigned)g.nprob);
    const size_t sh = (size_t)W * g.nz * sizeof(cx<T>);
    if (g.S <= 4)
        hipLaunchKernelGGL((k_z1<T, E, 4>), grid, dim3(NT), sh, s, g, a, W);
    else
        hipLaunchKernelGGL((k_z1<T, E, DFT_MAX_SPECIES>), grid, dim3(NT), sh, s, g, a, W);
    check_launch("z1");
}

template <typename T>
void launch_z2(const Geo &g, const Z2Args &a, hipStream_t s) {
    if (launch_z2_ct<T>(g, a, s)) return;
    if (g.compact) throw std::runtime_error("z2: compact vector layout without a compiled-length kernel");
    constexpr int E = Cfg<T>::ZE;
    const int W = yz_width<T, E>(g.nz, g.Kx);
    dim3 grid((unsigned)ceil_div(g.Kx, W), (unsigned)g.ny, (unsigned)g.nprob);
    const size_t sh = (size_t)W * g.nz * sizeof(cx<T>);
    hipLaunchKernelGGL((k_z2<T, E>), grid, dim3(NT), sh, s, g, a, W);
    check_launch("z2");
}

template <typename T>
int x3_nparts(const Geo &g) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    if (const int pb = x_ct_pairs(g.nx)) return (int)ceil_div(npairs, pb) * g.S;
    long long P = (NT * Cfg<T>::XE) / g.nx;
    if (P < 1) P = 1;
    if (P > npairs) P = npairs;
    return (int)ceil_div(npairs, P) * g.S;
}
template int x3_nparts<double>(const Geo &);
template int x3_nparts<float>(const Geo &);

int x3_blocks(const Geo &g) { return std::max(x3_nparts<double>(g), x3_nparts<float>(g)); }

// Batched x_fmt geometry: NTB threads, PB row pairs per block (10 PB nx <= NTB * 12),
// LDS of at most 64 KiB.  Returns false when the row is too long for it.
constexpr int kX2bE = 12;

template <typename T>
static bool x2b_geometry(const Geo &g, int *ntb, int *pb) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    for (int nt : {256, 512}) {
        int P = (nt * kX2bE) / (DFT_NALPHA * g.nx);
        if (P < 1) continue;
        if (P > npairs) P = (int)npairs;
        if ((size_t)DFT_NALPHA * P * g.nx * sizeof(cx<T>) > 65536) continue;
        *ntb = nt;
        *pb = P;
        return true;
    }
    return false;
}

template <typename T>
int x2_nblocks(const Geo &g) {
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    if (const int pb = x2_ct_min_pairs(g.nx)) return (int)ceil_div(npairs, pb);
    int ntb, pb;
    if (x2b_geometry<T>(g, &ntb, &pb)) return (int)ceil_div(npairs, pb);
    const int P = x_pairs<T, Cfg<T>::X2E>(g);
    return (int)ceil_div(npairs, P);
}

template <typename T>
int launch_x2(const Geo &g, const X2Args &a, hipStream_t s) {
    if (const int nb = launch_x2_ct<T>(g, a, s)) return nb;
    if (g.compact) throw std::runtime_error("x2: compact vector layout without a compiled-length kernel");
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    int ntb, pb;
    if (x2b_geometry<T>(g, &ntb, &pb)) {
        const long long nb = ceil_div(npairs, pb);
        if (nb > a.red.cap) throw std::runtime_error("x2: reduction buffer too small");
        const size_t sh = (size_t)DFT_NALPHA * pb * g.nx * sizeof(cx<T>);
        if (ntb == 256)
            hipLaunchKernelGGL((k_x2b<T, 256, kX2bE>), dim3((unsigned)nb, 1, (unsigned)g.nprob), dim3(256), sh, s, g, a,
                               pb);
        else
            hipLaunchKernelGGL((k_x2b<T, 512, kX2bE>), dim3((unsigned)nb, 1, (unsigned)g.nprob), dim3(512), sh, s, g, a,
                               pb);
        check_launch("x2b");
        return (int)nb;
    }
    if (a.mode == X2_HESS) throw std::runtime_error("x2: Hessian mode needs the batched kernel (n_x <= 384)");
    constexpr int E = Cfg<T>::X2E;
    const int P = x_pairs<T, E>(g);
    const long long nb = ceil_div(npairs, P);
    if (nb > a.red.cap) throw std::runtime_error("x2: reduction buffer too small");
    const size_t sh = (size_t)P * g.nx * sizeof(cx<T>);
    hipLaunchKernelGGL((k_x2<T, E>), dim3((unsigned)nb, 1, (unsigned)g.nprob), dim3(NT), sh, s, g, a, P);
    check_launch("x2");
    return (int)nb;
}

template int x2_nblocks<double>(const Geo &);
template int x2_nblocks<float>(const Geo &);

int x2_blocks(const Geo &g) { return std::max(x2_nblocks<double>(g), x2_nblocks<float>(g)); }

template <typename T>
void launch_x3(const Geo &g, const X3Args &a, hipStream_t s) {
    if (launch_x3_ct<T>(g, a, s)) return;
    constexpr int E = Cfg<T>::XE;
    const int P = x_pairs<T, E>(g);
    const long long npairs = ((long long)g.ny * g.nz + 1) / 2;
    const long long nb = ceil_div(npairs, P);
    if (!a.raw && nb * a.nfield > a.red.cap) throw std::runtime_error("x3: reduction buffer too small");
    dim3 grid((unsigned)nb, (unsigned)a.nfield, (unsigned)g.nprob);
    const size_t sh = (size_t)P * g.nx * sizeof(cx<T>);
    hipLaunchKernelGGL((k_x3<T, E>), grid, dim3(NT), sh, s, g, a, P);
    check_launch("x3");
}

template void launch_x_forward<double>(const Geo &, const XFwdArgs &, hipStream_t);
template void launch_x_forward<float>(const Geo &, const XFwdArgs &, hipStream_t);
template void launch_y<double>(const Geo &, const YArgs &, hipStream_t);
template void launch_y<float>(const Geo &, const YArgs &, hipStream_t);
template void launch_z1<double>(const Geo &, const Z1Args &, hipStream_t);
template void launch_z1<float>(const Geo &, const Z1Args &, hipStream_t);
template void launch_z2<double>(const Geo &, const Z2Args &, hipStream_t);
template void launch_z2<float>(const Geo &, const Z2Args &, hipStream_t);
template int launch_x2<double>(const Geo &, const X2Args &, hipStream_t);
template int launch_x2<float>(const Geo &, const X2Args &, hipStream_t);
template void launch_x3<double>(const Geo &, const X3Args &, hipStream_t);
template void launch_x3<float>(const Geo &, const X3Args &, hipStream_t);

// --------------------------------------------------------------------- reductions, control
// Reduction of the per-block partials of one evaluation into its state slots: 1024 threads,
// four independent accumulators per thread over fixed strides, then wave and block trees in
// fixed order, so the result is the same for every launch of the same shape.
constexpr int kNTF = 1024;

__global__ __launch_bounds__(kNTF) void k_finalize(RedBufs r, int nf, int nm, double *fslot, double *mslot,
                                                   DevState *st, int count_kind, const int *gate, long long pstride) {
    const long long off = (long long)blockIdx.x * pstride;
    gate = shp(gate, off);
    if (gated_off(gate)) return;
    r = shift(r, off);
    fslot = shp(fslot, off);
    mslot = shp(mslot, off);
    st = shp(st, off);
    __shared__ double ss[kNTF / 64], sm[kNTF / 64];
    __shared__ int sf[kNTF / 64];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    double m0 = -INFINITY, m1 = -INFINITY;
    int fl = 0;
    int b = t;
    for (; b + 3 * kNTF < nf; b += 4 * kNTF) {
        a0 += r.fpart[b];
        a1 += r.fpart[b + kNTF];
        a2 += r.fpart[b + 2 * kNTF];
        a3 += r.fpart[b + 3 * kNTF];
        fl |= r.fflag[b] | r.fflag[b + kNTF] | r.fflag[b + 2 * kNTF] | r.fflag[b + 3 * kNTF];
    }
    for (; b < nf; b += kNTF) {
        a0 += r.fpart[b];
        fl |= r.fflag[b];
    }
    b = t;
    for (; b + kNTF < nm; b += 2 * kNTF) {
        m0 = fmax(m0, r.mpart[b]);
        m1 = fmax(m1, r.mpart[b + kNTF]);
        fl |= r.mflag[b] | r.mflag[b + kNTF];
    }
    for (; b < nm; b += kNTF) {
        m0 = fmax(m0, r.mpart[b]);
        fl |= r.mflag[b];
    }
    double a = wave_sum((a0 + a1) + (a2 + a3));
    double m = wave_max(fmax(m0, m1));
    fl = wave_or(fl);
    const int w = t / 64;
    if (t % 64 == 0) {
        ss[w] = a;
        sm[w] = m;
        sf[w] = fl;
    }
    __syncthreads();
    if (t == 0) {
        double sa = ss[0], sx = sm[0];
        int sfl = sf[0];
        for (int i = 1; i < kNTF / 64; ++i) {
            sa += ss[i];
            sx = fmax(sx, sm[i]);
            sfl |= sf[i];
        }
        const bool bad = (sfl & 1) || !isfinite(sa);
        if (fslot) *fslot = bad ? INFINITY : sa;
        if (mslot) *mslot = (sfl & 4) ? INFINITY : sx;
        if (st) {
            if (count_kind == 1) st->gevals += 1;
            if (count_kind == 2) st->n3evals += 1;
        }
    }
}

void launch_finalize(const RedBufs &r, int nf, int nm, double *fslot, double *mslot, DevState *st, int count_kind,
                     const int *gate, hipStream_t s, int nprob, long long pstride) {
    hipLaunchKernelGGL(k_finalize, dim3(nprob), dim3(kNTF), 0, s, r, nf, nm, fslot, mslot, st, count_kind, gate,
                       pstride);
    check_launch("finalize");
}

constexpr double kCapFloor = 1.0 / 1024.0;

// Line-search state machine (one thread).  The order of samples and the acceptance rule
// follow the nonlinear-solver section as read in the oracle: samples at amax/2 and amax,
// quadratic fit in t = alpha / amax, best evaluated point accepted if it lowers f.
__global__ void k_ctl(DevState *st, int op, int nprob, long long pstride) {
    const int prob = blockIdx.x * blockDim.x + threadIdx.x;
    if (prob >= nprob) return;
    DevState &s = *shp(st, (long long)prob * pstride);
    switch (op) {
    case CTL_PRIME: {
        s.r = sqrt(s.f0 / s.nfluid);
        if (!isfinite(s.f0)) s.status = DFT_E_NONFINITE;
        s.converged = s.r <= s.tol ? 1 : 0;
        s.gate_run = (!s.converged && s.status == 0 && s.iters < s.max_iter) ? 1 : 0;
        s.gate_one = 1;
        s.alpha_zero = 0.0;
        s.alpha_one = 1.0;
        break;
    }
    case CTL_BEGIN: {
        int run = s.gate_run && s.status == 0 && !s.converged && s.iters < s.max_iter &&
                  s.rejected < 4 * s.max_iter + 16;
        if (run && !(s.m0 < s.eta_cap)) { s.status = DFT_E_PACKING; run = 0; }
        s.gate_run = run;
        s.gate_full1 = run && s.cap >= 1.0;
        s.gate_part1 = run && s.cap < 1.0;
        s.gate_a = run;
        s.gate_b = 0;
        s.gate_s = 0;
        s.alpha_trial = 1.0;
        break;
    }
    case CTL_AMAX: {
        if (!s.gate_run) break;
        const double bound = (s.m1 <= s.eta_cap) ? 1.0 : (s.eta_cap - s.m0) / (s.m1 - s.m0);
        s.amax = fmin(s.cap, bound);
        s.alpha_trial = 0.5 * s.amax;
        break;
    }
    case CTL_B: {
        if (!s.gate_run) break;
        s.gate_b = !(s.gate_full1 && s.amax == 1.0);
        if (!s.gate_b) { s.fb = s.f1; s.mb = s.m1; }
        s.alpha_trial = s.amax;
        break;
    }
    case CTL_FIT: {
        if (!s.gate_run) break;
        const double c2 = 2.0 * (s.f0 - 2.0 * s.fa + s.fb);
        const double c1 = s.fb - s.f0 - c2;
        double t;
        if (c2 > 0.0) t = fmin(fmax(-c1 / (2.0 * c2), 0.01), 1.0);
        else t = (s.fb <= s.fa) ? 1.0 : 0.5;
        s.t = t;
        s.gate_s = (t != 1.0 && t != 0.5);
        s.alpha_trial = t * s.amax;
        break;
    }
    case CTL_ACCEPT: {
        if (!s.gate_run) break;
        double bf = s.fb, bt = 1.0, bm = s.mb;
        int src = 0;
        if (s.fa < bf || (s.fa == bf && 0.5 > bt)) { bf = s.fa; bt = 0.5; bm = s.ma; src = 1; }
        if (s.gate_s && (s.fs < bf || (s.fs == bf && s.t > bt))) { bf = s.fs; bt = s.t; bm = s.ms; src = 2; }
        s.best_f = bf;
        if (bf < s.f0 || s.amax <= kCapFloor) {
            if (!isfinite(bf)) { s.status = DFT_E_NONFINITE; s.gate_run = 0; break; }
            s.alpha_acc = bt * s.amax;
            s.f0 = bf;
            s.m0 = bm;
            s.src = src;
            // the accepted sample's trial density (rho0 + alpha_acc (g0 - rho0), formed by the x
            // pass as the update would form it) and its image become the iterate: a role change
            s.sel = (s.sel + 1 + src) & 3;
            if (s.alpha_acc >= 0.5 * s.cap) s.cap = fmin(1.0, 2.0 * s.cap);
            s.iters += 1;
        } else {
            s.alpha_acc = 0.0;
            s.cap = fmax(0.25 * s.amax, kCapFloor);
            s.rejected += 1;
        }
        break;
    }
    case CTL_END: {
        s.r = sqrt(s.f0 / s.nfluid);
        s.converged = s.r <= s.tol ? 1 : 0;
        s.gate_run = (s.gate_run && !s.converged && s.status == 0 && s.iters < s.max_iter) ? 1 : 0;
        break;
    }
    }
}

void launch_ctl(DevState *st, int op, hipStream_t s, int nprob, long long pstride) {
    hipLaunchKernelGGL(k_ctl, dim3((nprob + 63) / 64), dim3(64), 0, s, st, op, nprob, pstride);
    check_launch("ctl");
}

struct BaseArgs {
    double mu[DFT_MAX_SPECIES];
    double z[DFT_MAX_SPECIES];
};

__global__ __launch_bounds__(NT) void k_make_base(int S, long long N, const double *vext, const double *phi,
                                                  double *base, BaseArgs ba, double *count_part) {
    double cnt = 0.0;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < (long long)S * N; t += (long long)gridDim.x * NT) {
        const int i = (int)(t / N);
        const long long x = t - (long long)i * N;
        const double v = vext ? vext[t] : 0.0;
        double b = -INFINITY;
        if (isfinite(v)) {
            b = ba.mu[i] - v;
            if (phi) b -= ba.z[i] * phi[x];
            cnt += 1.0;
        } else if (isnan(v)) {
            b = NAN;
        }
        base[t] = b;
    }
    __shared__ double sc[NT];
    sc[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sc[threadIdx.x] += sc[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) count_part[blockIdx.x] = sc[0];
}

void launch_make_base(const Consts *, int S, long long N, const double *vext, const double *phi_fixed, double *base,
                      const double *mu_host, const double *z_host, double *count_part, int nblk, hipStream_t s) {
    BaseArgs ba;
    for (int i = 0; i < DFT_MAX_SPECIES; ++i) {
        ba.mu[i] = i < S ? mu_host[i] : 0.0;
        ba.z[i] = i < S ? z_host[i] : 0.0;
    }
    hipLaunchKernelGGL(k_make_base, dim3(nblk), dim3(NT), 0, s, S, N, vext, phi_fixed, base, ba, count_part);
    check_launch("make_base");
}

__global__ __launch_bounds__(NT) void k_sum_to(const double *part, int n, double *dst) {
    __shared__ double sc[NT];
    double a = 0.0;
    for (int b = threadIdx.x; b < n; b += NT) a += part[b];
    sc[threadIdx.x] = a;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sc[threadIdx.x] += sc[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dst = sc[0];
}

void launch_sum_to(const double *part, int n, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(NT), 0, s, part, n, dst);
    check_launch("sum_to");
}

__global__ __launch_bounds__(NT) void k_copy(double *dst, const double *src, long long n, long long pstride,
                                             const int *gate) {
    const long long off = (long long)blockIdx.y * pstride;
    if (gated_off(shp(gate, off))) return;
    dst = shp(dst, off);
    src = shp(src, off);
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) dst[i] = src[i];
}

__global__ __launch_bounds__(NT) void k_copy_current(double *dst, Roles roles, long long n, long long pstride,
                                                     const int *gate) {
    const long long off = (long long)blockIdx.y * pstride;
    if (gated_off(shp(gate, off))) return;
    dst = shp(dst, off);
    roles = shift(roles, off);
    const double *src = role_pick(roles.rho, role_sel(roles.sel));
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) dst[i] = src[i];
}

void launch_copy_current(double *dst, const Roles &roles, long long count, hipStream_t s, int nprob,
                         long long pstride, const int *gate) {
    const long long nb = std::min<long long>(ceil_div(count, NT), 8192);
    hipLaunchKernelGGL(k_copy_current, dim3((unsigned)nb, (unsigned)nprob), dim3(NT), 0, s, dst, roles, count, pstride,
                       gate);
    check_launch("copy current");
}

void launch_copy(double *dst, const double *src, long long count, hipStream_t s, int nprob, long long pstride,
                 const int *gate) {
    const long long nb = std::min<long long>(ceil_div(count, NT), 8192);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)nb, (unsigned)nprob), dim3(NT), 0, s, dst, src, count, pstride, gate);
    check_launch("copy");
}

// Copies nrec line-search state records between strided places (byte strides): gathers the
// states of a batch group's problems into one contiguous array for a single host read, and
// writes them back.  With `gates`, only gate_refresh of every record is written, from gates[i].
__global__ __launch_bounds__(NT) void k_copy_states(char *dst, long long dst_stride, const char *src,
                                                    long long src_stride, int nrec, const int *gates) {
    const int rec = blockIdx.x;
    if (rec >= nrec) return;
    DevState *d = reinterpret_cast<DevState *>(dst + rec * dst_stride);
    if (gates) {
        if (threadIdx.x == 0) d->gate_refresh = gates[rec];
        return;
    }
    constexpr int W = (int)(sizeof(DevState) / sizeof(int));
    static_assert(sizeof(DevState) % sizeof(int) == 0, "state record is not a whole number of ints");
    const int *s = reinterpret_cast<const int *>(src + rec * src_stride);
    int *dd = reinterpret_cast<int *>(d);
    for (int i = threadIdx.x; i < W; i += NT) dd[i] = s[i];
}

void launch_copy_states(void *dst, long long dst_stride, const void *src, long long src_stride, int nrec,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_copy_states, dim3((unsigned)nrec), dim3(NT), 0, s, (char *)dst, dst_stride,
                       (const char *)src, src_stride, nrec, (const int *)nullptr);
    check_launch("copy_states");
}

void launch_set_gates(DevState *first, long long stride, int nrec, const int *gates, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_states, dim3((unsigned)nrec), dim3(NT), 0, s, (char *)first, stride,
                       (const char *)nullptr, 0LL, nrec, gates);
    check_launch("set_gates");
}

}  // namespace dft
