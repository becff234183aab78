// Pass kernels with the transform length fixed at compile time (fft_ct.h).  They compute
// the same transforms as the run-time-length kernels, and every launch shape of one length
// (tile width, threads, LDS buffering) performs the same arithmetic in the same order, so
// the choice among shapes never changes a result.
#pragma once

#include <stdexcept>
#include <string>
#include <type_traits>
#include <utility>

#include "dft_kernels.h"
#include "fft_ct.h"
#include "pass_util.h"

namespace dft {

// Threads per block: a power of two in [64, cap] near L P / per (per = values per thread).
constexpr int fit_threads(int L, int P, int per, int cap) {
    int t = 64;
    while (2 * t <= cap && 2 * t * per <= L * P) t *= 2;
    return t;
}

inline void ct_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

inline long long ct_cdiv(long long a, long long b) { return (a + b - 1) / b; }

// f(integral_constant<int, i>) for i = 0..N-1: a loop whose index is a constant in every body,
// whatever the body's size (register arrays indexed by it stay in registers).
template <class Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

#define DFT_CT_LENGTHS(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384)

// ------------------------------------------------------------------ y / z plain transforms
// One block transforms P adjacent pencils of one field along y or z; the pencils' elements sit
// rs apart in HBM, and adjacent pencils of one row are adjacent in HBM.
// VEC = 1, 2: the y passes of the compact vector layout (Geo::compact), where a block of the
// n3 or nV1-sum slot makes two transforms (inverse: the field and -i k_y times it) and a block
// of a vector-derivative slot adds i k_y times the transform of the y component (forward).
template <typename T, int L, int P, int NTB, int NB, int VEC>
__global__ __launch_bounds__(NTB) void k_yc(Geo g_in, YArgs a) {
    using F = ct::Fft<T, typename ct::PlanT<T, L>::type, P, NTB, false, NB>;
    // blocks per problem: one per field, or per block type of the compact vector layout
    // (VEC = YArgs::vec, a template parameter so that the plain transforms keep their registers)
    const int ntypes = VEC == 1 ? 7 : (VEC == 2 ? 8 : a.nfield);
    const int prob = (int)blockIdx.z / ntypes;
    if (prob > 0) {
        const long long off = (long long)prob * g_in.pstride;
        g_in = shift(g_in, off);
        a = shift(a, off);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    __shared__ cx<T> lds[F::LDS_ELEMS];
    const bool zax = a.axis == 2;
    const int Kx = g.Kx;
    // A tile is P consecutive pencils of the flattened plane of pencils, (y, kx) as y Kx + kx for
    // the z axis (as in the other z tiles), (z, kx) as z Kx + kx for the y axis, so no tile holds
    // a lone Nyquist column.  A thread keeps one pencil (p = threadIdx.x mod P) and its offset.
    static_assert(NTB % P == 0, "a thread keeps one pencil");
    int bx, unused;
    xcd_block(bx, unused);
    const int ncol = (zax ? g.ny : g.nz) * Kx;
    const int c0 = bx * P;
    const int Pact = min(P, ncol - c0);
    const int col = min(c0 + (int)threadIdx.x % P, ncol - 1);
    const int zc = zax ? 0 : col / Kx;
    const int jx = col - zc * Kx;   // k_x index of the pencil (y axis)
    const int f = (int)blockIdx.z % ntypes;
    const long long rs = zax ? (long long)g.ny * Kx : (long long)Kx;
    cx<T> *spec = reinterpret_cast<cx<T> *>(a.spec) + (zax ? (long long)col : (long long)zc * g.ny * Kx + jx);
    const cx<T> *tw = twp<T>(g, zax ? 2 : 1);
    // grid steps of k_x, k_y read before any store (read later they would be reloaded after each)
    [[maybe_unused]] const T dkx = T(g.cs->dk[0]), dky = T(g.cs->dk[1]);
    cx<T> v[F::V];
    int ph = 0;
    auto body = [&](auto dirc) {
        constexpr int DIR = decltype(dirc)::value;
        auto load = [&](int slot, cx<T> *w) {
            const cx<T> *base = spec + (long long)slot * g.NC;
#pragma unroll
            for (int i = 0; i < F::template nin<DIR>(); ++i) {
                int p, e;
                const bool ok = F::template in_pos<DIR>(i, p, e);
                w[i] = (ok && p < Pact) ? ct::gld(base + e * rs) : mk<T>(T(0), T(0));
            }
        };
        // store slot, times -i k_x when mx (k_x of the column, zero on the Nyquist column)
        auto store = [&](int slot, const cx<T> *w, bool mx) {
            cx<T> *base = spec + (long long)slot * g.NC;
#pragma unroll
            for (int i = 0; i < F::template nout<DIR>(); ++i) {
                int p, e;
                const bool ok = F::template out_pos<DIR>(i, p, e);
                if (!(ok && p < Pact)) continue;
                cx<T> u = w[i];
                if (mx) {
                    const T kx = (g.nx % 2 == 0 && 2 * jx == g.nx) ? T(0) : T(jx) * dkx;
                    u = mk<T>(kx * u.y, -kx * u.x);
                }
                ct::gst(base + e * rs, u);
            }
        };
        // k_y of element e of the pencil (zero on the Nyquist row)
        auto ky = [&](int e) {
            return (g.ny % 2 == 0 && 2 * e == g.ny) ? T(0) : T(signed_mode(e, g.ny)) * dky;
        };
        if constexpr (VEC == 0) {
            load(f, v);
            F::template run<DIR>(v, lds, ph, tw);
            store(f, v, false);
        } else if constexpr (VEC == 1) {
            // inverse: slots 0-3 (n0..n3), 4 (nV1 sum), 6, 9 (z components) -> nine fields:
            // n3 also gives nV2_y = -i k_y n3, the nV1 sum gives nV1_x and nV1_y (slot 7,
            // nV2_x, is left to the x pass)
            const int slot = f < 5 ? f : (f == 5 ? 6 : 9);
            load(slot, v);
            if (slot == 3 || slot == 4) {
                cx<T> w[F::V];
#pragma unroll
                for (int i = 0; i < F::template nin<DIR>(); ++i) {
                    int p, e;
                    F::template in_pos<DIR>(i, p, e);
                    const T k = ky(e);
                    w[i] = mk<T>(k * v[i].y, -k * v[i].x);   // -i k_y
                }
                F::template run<DIR>(v, lds, ph, tw);
                store(slot, v, slot == 4);   // (n_V2,x = -i k_x n3 is formed by the x pass)
                F::template run<DIR>(w, lds, ph, tw);
                store(slot == 3 ? 8 : 5, w, false);
            } else {
                F::template run<DIR>(v, lds, ph, tw);
                store(slot, v, false);
            }
        } else {
            // forward: ten fields -> slots 0-3, 4 (i k_x dPhi_V1x + i k_y dPhi_V1y), 6, 7 (the same
            // for V2), 9; the x parts arrive multiplied by i k_x
            const int slot = f < 5 ? f : (f == 5 ? 6 : (f == 6 ? 7 : 9));
            load(slot, v);
            F::template run<DIR>(v, lds, ph, tw);
            if (slot == 4 || slot == 7) {
                cx<T> w[F::V];
                load(slot + 1, w);
                F::template run<DIR>(w, lds, ph, tw);
#pragma unroll
                for (int i = 0; i < F::template nout<DIR>(); ++i) {
                    int p, e;
                    F::template out_pos<DIR>(i, p, e);
                    const T k = ky(e);
                    v[i] = mk<T>(v[i].x - k * w[i].y, v[i].y + k * w[i].x);   // + i k_y w
                }
            }
            store(slot, v, false);
        }
    };
    if (a.dir < 0) body(std::integral_constant<int, -1>());
    else body(std::integral_constant<int, 1>());
}

// ------------------------------------------------------------------ z passes
// z tiles run over the plane of columns (y, kx) flattened as y Kx + kx: a tile is P consecutive
// columns, whatever row they fall in, so a plane of n_y Kx columns needs ceil(n_y Kx / P) tiles
// (none holding a lone Nyquist column) and, with n_y Kx a multiple of P, every tile's segment of
// a z plane starts on a P-element boundary.  In these tiles (pencil index fastest over threads,
// NTB a multiple of P) a thread keeps one column, p = threadIdx.x mod P.
struct ZTile {
    long long off;   // first column of the tile (offset of its segment in a z plane)
    int Pact;        // columns of the tile inside the plane
    int x, y;        // the thread's column (a valid column also for idle lanes of a ragged tile)
};
template <int P>
__device__ __forceinline__ ZTile z_tile(const Geo &g) {
    int t, unused;
    xcd_block(t, unused);
    const int ncol = g.ny * g.Kx;
    const int c0 = t * P;
    ZTile z;
    z.off = c0;
    z.Pact = min(P, ncol - c0);
    const int col = min(c0 + (int)threadIdx.x % P, ncol - 1);
    z.y = col / g.Kx;
    z.x = col - z.y * g.Kx;
    return z;
}

// Wavenumbers of the elements of one z pencil: column (x, y), z index e.  Only the indices are
// kept per thread (the grid steps are uniform): the components are formed at each use, which
// costs a few instructions and no registers across the transforms.
template <typename T>
struct ZWave {
    T dkx, dky, dkz;
    int x, y, nx, ny, nz;
    __device__ __forceinline__ ZWave(const Consts &c, int x_, int y_) : x(x_), y(y_) {
        dkx = T(c.dk[0]);
        dky = T(c.dk[1]);
        dkz = T(c.dk[2]);
        nx = c.nx;
        ny = c.ny;
        nz = c.nz;
    }
    __device__ __forceinline__ T kx() const { return T(x) * dkx; }
    __device__ __forceinline__ T ky() const { return T(signed_mode(y, ny)) * dky; }
    __device__ __forceinline__ T kz(int e) const { return T(signed_mode(e, nz)) * dkz; }
    __device__ __forceinline__ T kmag(int e) const {
        const T a = kx(), b = ky(), d = kz(e);
        return sqrt_r(a * a + b * b + d * d);
    }
    __device__ __forceinline__ bool zero(int e) const { return x == 0 && y == 0 && e == 0; }
    // component d of k, zero on the Nyquist plane of axis d
    __device__ __forceinline__ T comp(int e, int d) const {
        if (d == 0) return ((nx % 2 == 0) && 2 * x == nx) ? T(0) : kx();
        if (d == 1) return ((ny % 2 == 0) && 2 * y == ny) ? T(0) : ky();
        return ((nz % 2 == 0) && 2 * e == nz) ? T(0) : kz(e);
    }
};

// Eigenvalue of minus the 7-point Laplacian, sum_d 4 sin^2(k_d h_d / 2) / h_d^2, from the
// twiddle tables: k_d h_d = 2 pi j_d / n_d, and tw_d[j] = exp(-2 pi i j / n_d).  The x and y
// terms are those of one column (x, y).
template <typename T>
struct Poisson {
    const cx<T> *tz;
    T ih2z, dxy;
    __device__ __forceinline__ Poisson() : tz(nullptr), ih2z(0), dxy(0) {}
    __device__ __forceinline__ Poisson(const Geo &g, const Consts &c, int x, int y) {
        tz = twp<T>(g, 2);
        ih2z = T(1.0 / (c.h[2] * c.h[2]));
        const cx<T> wx = ct::cld(twp<T>(g, 0) + x), wy = ct::cld(twp<T>(g, 1) + y);
        dxy = two_omc<T>(wx.x, wx.y) * T(1.0 / (c.h[0] * c.h[0])) + two_omc<T>(wy.x, wy.y) * T(1.0 / (c.h[1] * c.h[1]));
    }
    __device__ __forceinline__ T denom(int e) const {
        const cx<T> wz = ct::cld(tz + e);
        return dxy + two_omc<T>(wz.x, wz.y) * ih2z;
    }
};

// Pair row of the spectral table (rows [row][z][y][kx], see Geo::tab64): K_ij, i <= j.
__device__ __forceinline__ int pair_row(int S, int i, int j) {
    const int a = min(i, j), b = max(i, j);
    return 2 * S + a * S - (a * (a - 1)) / 2 + (b - a);
}

// Z1: forward z transform of every species, then per element
//   (a) the five weighted sums of Appendix B spectra giving the ten n_alpha spectra (the
//       vector spectra are -i k times a w3 sum), each inverse z transformed into specB;
//   (b) with electrostatics (MS > 0 bounds S), per species i the linear electrostatic part
//       of the exponent sum_j K_ij(k) (rho_hat_j - N rho_b_j delta_k0), K_ij = C_ij(k) -
//       z_i z_j 4 pi l_B / D(k) (eqs. muESexpansion, potentialSolution), written
//       unnormalized over rho_hat in specA (z spectral order).
// FP64 takes the spectral factors from the setup-time tables; FP32 (differences from the
// reference) evaluates them on the fly: sin and cos of k R once per species, the pair
// terms by the addition theorem, the Poisson denominator from the twiddle tables -- in
// FP32 that is cheaper than moving the tables.  The products act on registers between
// the forward and inverse transforms.  Every Z1 kernel (fused or split, any tile width) does
// the same arithmetic in the same order, so the autotuner's choice does not change a result.

// Slot of the unordered species pair a <= b < MS.
template <int MS>
__device__ __forceinline__ constexpr int pair_slot(int a, int b) {
    return a * MS - (a * (a - 1)) / 2 + (b - a);
}

// The species and pair constants of the products in the arithmetic type, read once per block
// before any store (read at their uses they would be reloaded and converted after every store,
// which may alias them).  Pair p = pair_slot(a, b), a <= b.
template <typename T, int MS>
struct Z1Const {
    static constexpr int NPR = MS * (MS + 1) / 2;
    T R[MS], a0[MS], a1[MS], bath[MS];   // R_j, 1 / (4 pi R_j^2), 1 / (4 pi R_j), N rho_b,j
    T zz[NPR], scR[NPR], p1[NPR], p2[NPR], p3[NPR], p4[NPR];   // pair constants (FP32 only)
    T four_pi_lB;
    __device__ __forceinline__ explicit Z1Const(const Consts &c) {
        constexpr bool F32 = std::is_same<T, float>::value;
        static_for<MS>([&](auto J) __attribute__((always_inline)) {
            constexpr int j = J;
            if constexpr (F32) {
                R[j] = c.f_R[j];
                a0[j] = c.f_i4piR2[j];
                a1[j] = c.f_i4piR[j];
                bath[j] = c.f_bath_N[j];
            } else {
                R[j] = c.R[j];
                a0[j] = c.i4piR2[j];
                a1[j] = c.i4piR[j];
                bath[j] = c.bath_N[j];
            }
        });
        static_for<MS>([&](auto IA) __attribute__((always_inline)) {
            static_for<MS>([&](auto IB) __attribute__((always_inline)) {
                constexpr int ia = IA, ib = IB;
                if constexpr (ib >= ia) {
                    constexpr int q = pair_slot<MS>(ia, ib), ij = ia * DFT_MAX_SPECIES + ib;
                    if constexpr (F32) {
                        zz[q] = c.f_zz[ij];
                        scR[q] = c.f_sc_R[ij];
                        p1[q] = c.f_sc_p1[ij];
                        p2[q] = c.f_sc_p2[ij];
                        p3[q] = c.f_sc_p3[ij];
                        p4[q] = c.f_sc_p4[ij];
                    } else {
                        // FP64 reads the pair factors from the spectral tables
                        zz[q] = c.z[ia] * c.z[ib];
                        scR[q] = p1[q] = p2[q] = p3[q] = p4[q] = T(0);
                    }
                }
            });
        });
        four_pi_lB = F32 ? c.f_four_pi_lB : c.four_pi_lB;
    }
};

// Products of one node with electrostatics (S <= MS): the species values u at the node (k_x
// column p of the tile, z element e; ti its offset in a spectrum, ok whether it is a real
// column), the five weighted sums out in acc, and the node's sums over j of K_ij times the
// species spectra stored at dst + i NC.  Each unordered pair factor is formed once (K_ij = K_ji).
template <typename T, int MS>
__device__ __forceinline__ void z1_node(const Z1Const<T, MS> &k, bool diff, const ZWave<T> &kw, const Poisson<T> &pd,
                                        const double *tab, long long NC, int S, bool es, int e, bool ok,
                                        long long ti, const cx<T> (&u)[MS], cx<T> (&acc)[5], cx<T> *dst) {
    constexpr bool TAB = std::is_same<T, double>::value;
    constexpr int NPR = MS * (MS + 1) / 2;
    T w2[MS], w3[MS], K[NPR];
    // every loop over species or pairs has constant indices (static_for), whatever its size
    if constexpr (TAB) {
        static_for<MS>([&](auto J) __attribute__((always_inline)) {
            constexpr int j = J;
            w2[j] = (ok && j < S) ? ct::cld(tab + (long long)j * NC + ti) : T(0);
            w3[j] = (ok && j < S) ? ct::cld(tab + (long long)(S + j) * NC + ti) : T(0);
        });
        static_for<MS>([&](auto IA) __attribute__((always_inline)) {
            static_for<MS>([&](auto IB) __attribute__((always_inline)) {
                constexpr int ia = IA, ib = IB;
                if constexpr (ib >= ia)
                    K[pair_slot<MS>(ia, ib)] =
                        (ok && es && ib < S) ? ct::cld(tab + (long long)pair_row(S, ia, ib) * NC + ti) : T(0);
            });
        });
    } else {
        const T km = kw.kmag(e);
        T sn[MS], cs[MS];
        static_for<MS>([&](auto J) __attribute__((always_inline)) {
            constexpr int j = J;
            sn[j] = T(0);
            cs[j] = T(1);
            w2[j] = w3[j] = T(0);
            if (j < S) {
                sincos_w(km * k.R[j], &sn[j], &cs[j]);
                weight_w2_w3_sc<T>(km, k.R[j], sn[j], cs[j], w2[j], w3[j]);
            }
        });
        static_for<MS>([&](auto IA) __attribute__((always_inline)) {
            static_for<MS>([&](auto IB) __attribute__((always_inline)) {
                constexpr int ia = IA, ib = IB;
                if constexpr (ib >= ia) {
                    T Kv = T(0);
                    if (es && ib < S) {
                        // sin, cos of k (R_a + R_b) by the addition theorem: the contact cutoff (the
                        // launcher sends the cutoff at lambda_a + lambda_b to the run-time-length kernel)
                        const T sp = sn[ia] * cs[ib] + cs[ia] * sn[ib];
                        const T cp = cs[ia] * cs[ib] - sn[ia] * sn[ib];
                        constexpr int q = pair_slot<MS>(ia, ib);
                        Kv = screening_hat_p<T>(km, k.scR[q], sp, cp, k.p1[q], k.p2[q], k.p3[q], k.p4[q]);
                    }
                    K[pair_slot<MS>(ia, ib)] = Kv;
                }
            });
        });
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) acc[m] = mk<T>(T(0), T(0));
    static_for<MS>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = J;
        if (j < S) {
            const T a0 = k.a0[j], a1 = k.a1[j];
            const T m0 = w2[j] * a0, m1 = w2[j] * a1, m4 = w3[j] * a1;
            acc[0].x += u[j].x * m0; acc[0].y += u[j].y * m0;
            acc[1].x += u[j].x * m1; acc[1].y += u[j].y * m1;
            acc[2].x += u[j].x * w2[j]; acc[2].y += u[j].y * w2[j];
            acc[3].x += u[j].x * w3[j]; acc[3].y += u[j].y * w3[j];
            acc[4].x += u[j].x * m4; acc[4].y += u[j].y * m4;
        }
    });
    if (!(es && ok)) return;
    // the bath term enters the k = 0 element of the pair-correlation part only
    const bool z0 = !diff && kw.zero(e);
    T invD = T(0);
    if constexpr (!TAB)
        if (!kw.zero(e)) invD = k.four_pi_lB * rcp_r(pd.denom(e));
    static_for<MS>([&](auto IS) __attribute__((always_inline)) {
        constexpr int is = IS;
        if (is < S) {
            cx<T> ea = mk<T>(T(0), T(0));
            static_for<MS>([&](auto J) __attribute__((always_inline)) {
                constexpr int j = J;
                if (j < S) {
                    constexpr int q = is <= j ? pair_slot<MS>(is, j) : pair_slot<MS>(j, is);
                    const T Kij = K[q];
                    const T ux = z0 ? u[j].x - k.bath[j] : u[j].x;
                    if constexpr (TAB) {
                        ea.x += Kij * ux;
                        ea.y += Kij * u[j].y;
                    } else {
                        const T Pz = invD * k.zz[q];
                        ea.x += Kij * ux - Pz * u[j].x;
                        ea.y += (Kij - Pz) * u[j].y;
                    }
                }
            });
            ct::gst(dst + (long long)is * NC, ea);
        }
    });
}

// Products of one species at one node without electrostatics (species by species).
template <typename T>
__device__ __forceinline__ void z1_species(const Consts &c, const ZWave<T> &kw, const double *tab, long long NC, int S,
                                           int jsp, int e, bool ok, long long ti, cx<T> u, cx<T> (&acc)[5]) {
    T w2, w3;
    if constexpr (std::is_same<T, double>::value) {
        w2 = ok ? ct::cld(tab + (long long)jsp * NC + ti) : T(0);
        w3 = ok ? ct::cld(tab + (long long)(S + jsp) * NC + ti) : T(0);
    } else {
        weight_w2_w3<T>(kw.kmag(e), T(c.R[jsp]), w2, w3);
    }
    const T a0 = T(c.i4piR2[jsp]), a1 = T(c.i4piR[jsp]);
    const T m0 = w2 * a0, m1 = w2 * a1, m4 = w3 * a1;
    acc[0].x += u.x * m0; acc[0].y += u.y * m0;
    acc[1].x += u.x * m1; acc[1].y += u.y * m1;
    acc[2].x += u.x * w2; acc[2].y += u.y * w2;
    acc[3].x += u.x * w3; acc[3].y += u.y * w3;
    acc[4].x += u.x * m4; acc[4].y += u.y * m4;
}

// The seven inverse transforms of Z1 and their stores.  Along a z pencil k_x and k_y are
// constant, so the x and y components of the vector densities are -i k_x and -i k_y times the
// transform of their scalar sum; only n0..n3, the two vector sums' k_z multiples and the nV1 sum
// are transformed.  Transform t, its source sum and whether it is multiplied by -i k_z:
//   t = 0..3: acc[t] (n0..n3; t = 3 also gives the x, y components of nV2)
//   t = 4: acc[4] (x, y components of nV1);  t = 5: -i k_z acc[4] (nV1_z);  t = 6: -i k_z acc[3] (nV2_z)
template <typename T, class F, int NO>
__device__ __forceinline__ void z1_inverse(const Geo &g, const Z1Args &a, const ZWave<T> &kw, cx<T> *lds, int &ph,
                                           const cx<T> *tw, int Pact, long long rs, long long off,
                                           const cx<T> (&acc)[NO][5]) {
    const Consts &c = *g.cs;
    const long long NC = g.NC;
    const int ntr = a.n3only ? 1 : 7;
    const T invN = T(c.invN);
    cx<T> v[F::V];
    typename F::template TwReg<1> tri;   // inverse twiddles, shared by the output transforms
    F::template load_tw<1>(tri, tw);
    for (int t = 0; t < ntr; ++t) {
        const int src = a.n3only ? 3 : (t < 5 ? t : (t == 5 ? 4 : 3));
        const bool kzm = t >= 5;
#pragma unroll
        for (int i = 0; i < NO; ++i) {
            // source sum selected with compile-time register indices
            cx<T> sm = acc[i][3];
#pragma unroll
            for (int m = 0; m < 5; ++m)
                if (m == src) sm = acc[i][m];
            if (kzm) {
                int p, e;
                F::template in_pos<1>(i, p, e);
                const T kd = kw.comp(e, 2);
                sm = mk<T>(kd * sm.y, -kd * sm.x);   // -i k_z s
            }
            v[i] = mk<T>(sm.x * invN, sm.y * invN);
        }
        F::template run<1>(v, lds, ph, tri);
        // store the transform as output o, times -i k_d for d = 0 (x) or 1 (y), plain for d < 0
        auto store = [&](int o, int d) {
            cx<T> *dst = reinterpret_cast<cx<T> *>(a.specB) + (long long)o * NC + off;
#pragma unroll
            for (int i = 0; i < F::template nout<1>(); ++i) {
                int p, e;
                const bool ok = F::template out_pos<1>(i, p, e);
                if (!(ok && p < Pact)) continue;
                cx<T> w = v[i];
                if (d >= 0) {
                    const T kd = kw.comp(e, d);
                    w = mk<T>(kd * w.y, -kd * w.x);
                }
                ct::gst(dst + e * rs + p, w);
            }
        };
        if (a.n3only) {
            store(0, -1);
        } else if (g.compact) {
            // compact layout: n0..n3, the nV1 sum, nV1_z, nV2_z (the inverse y pass expands)
            store(t < 5 ? t : (t == 5 ? 6 : 9), -1);
        } else if (t < 4) {
            store(t, -1);
            if (t == 3) {
                store(7, 0);
                store(8, 1);
            }
        } else if (t == 4) {
            store(4, 0);
            store(5, 1);
        } else {
            store(t == 5 ? 6 : 9, -1);
        }
    }
}

template <typename T, int L, int P, int NTB, int MS>
__global__ __launch_bounds__(NTB) void k_z1c(Geo g_in, Z1Args a) {
    using F = ct::Fft<T, typename ct::PlanT<T, L>::type, P, NTB, false, 2>;
    constexpr int NO = F::template nout<-1>();
    static_assert(NO == F::template nin<1>(), "inverse must start where the forward ends");
    constexpr bool TAB = std::is_same<T, double>::value;
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    __shared__ cx<T> lds[F::LDS_ELEMS];
    const Consts &c = *g.cs;
    const int Kx = g.Kx, S = g.S;
    const long long NC = g.NC;
    static_assert(NTB % P == 0, "a thread keeps one column");
    const ZTile zt = z_tile<P>(g);
    const int Pact = zt.Pact;
    const long long rs = (long long)g.ny * Kx;
    const long long off = zt.off;
    const cx<T> *tw = twp<T>(g, 2);
    const bool es = MS > 0 && c.es && !a.n3only;
    const ZWave<T> kw(c, zt.x, zt.y);
    // the products' constants, read before the first store
    [[maybe_unused]] const Z1Const<T, (MS > 0 ? MS : 1)> kc(c);
    const double *tab = TAB ? g.tab64 + off : nullptr;
    cx<T> acc[NO][5];
    cx<T> v[F::V];
    int ph = 0;
    typename F::template TwReg<-1> trs;   // forward twiddles, shared by the species transforms
    F::template load_tw<-1>(trs, tw);
    // each species' inputs are fetched while the previous species transforms
    constexpr int NIN = F::template nin<-1>();
    cx<T> vin[NIN];
    auto load_species = [&](int jsp) {
        const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specA) + (long long)jsp * NC + off;
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            int p, e;
            const bool ok = F::template in_pos<-1>(i, p, e);
            vin[i] = (ok && p < Pact) ? ct::gld(src + e * rs + p) : mk<T>(T(0), T(0));
        }
    };
    load_species(0);
    if constexpr (MS == 0) {
#pragma unroll
        for (int i = 0; i < NO; ++i)
#pragma unroll
            for (int m = 0; m < 5; ++m) acc[i][m] = mk<T>(T(0), T(0));
        for (int jsp = 0; jsp < S; ++jsp) {
#pragma unroll
            for (int i = 0; i < NIN; ++i) v[i] = vin[i];
            if (jsp + 1 < S) load_species(jsp + 1);
            F::template run<-1>(v, lds, ph, trs);
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                int p, e;
                const bool ok = F::template out_pos<-1>(i, p, e) && p < Pact;
                z1_species<T>(c, kw, tab, NC, S, jsp, e, ok, ok ? e * rs + p : 0, v[i], acc[i]);
            }
        }
    } else {
        // all species transformed first (S <= MS), then the products node by node
        cx<T> us[MS][NO];
        static_for<MS>([&](auto J) __attribute__((always_inline)) {
            constexpr int jsp = J;
#pragma unroll
            for (int i = 0; i < NO; ++i) us[jsp][i] = mk<T>(T(0), T(0));
            if (jsp < S) {
#pragma unroll
                for (int i = 0; i < NIN; ++i) v[i] = vin[i];
                if (jsp + 1 < S) load_species(jsp + 1);
                F::template run<-1>(v, lds, ph, trs);
#pragma unroll
                for (int i = 0; i < NO; ++i) us[jsp][i] = v[i];
            }
        });
        Poisson<T> pd;
        if constexpr (!TAB) pd = Poisson<T>(g, c, zt.x, zt.y);
        static_for<NO>([&](auto I) __attribute__((always_inline)) {
            constexpr int i = I;
            int p, e;
            const bool ok = F::template out_pos<-1>(i, p, e) && p < Pact;
            const long long ti = ok ? e * rs + p : 0;
            cx<T> u[MS];
#pragma unroll
            for (int j = 0; j < MS; ++j) u[j] = us[j][i];
            z1_node<T, MS>(kc, a.diff != 0, kw, pd, tab, NC, S, es, e, ok, ti, u, acc[i],
                           reinterpret_cast<cx<T> *>(a.specA) + off + ti);
        });
    }
    z1_inverse<T, F, NO>(g, a, kw, lds, ph, tw, Pact, rs, off, acc);
}

// Z1 from z spectra: the same products and inverse transforms as k_z1c, for species spectra
// that the plain z pass has already transformed along z (the autotuner's split Z1 shapes).  With
// the forward transform in its own kernel, this one needs neither the prefetched inputs nor the
// forward twiddles in registers.  Each thread reads the species values at the positions it
// starts the inverse transforms from and overwrites them with the electrostatic spectra only
// after reading them.
template <typename T, int L, int P, int NTB, int MS>
__global__ __launch_bounds__(NTB) void k_z1s(Geo g_in, Z1Args a) {
    using F = ct::Fft<T, typename ct::PlanT<T, L>::type, P, NTB, false, 2>;
    constexpr int NO = F::template nin<1>();
    constexpr bool TAB = std::is_same<T, double>::value;
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    __shared__ cx<T> lds[F::LDS_ELEMS];
    const Consts &c = *g.cs;
    const int Kx = g.Kx, S = g.S;
    const long long NC = g.NC;
    static_assert(NTB % P == 0, "a thread keeps one column");
    const ZTile zt = z_tile<P>(g);
    const int Pact = zt.Pact;
    const long long rs = (long long)g.ny * Kx;
    const long long off = zt.off;
    const cx<T> *tw = twp<T>(g, 2);
    const bool es = MS > 0 && c.es && !a.n3only;
    const ZWave<T> kw(c, zt.x, zt.y);
    // the products' constants, read before the first store
    [[maybe_unused]] const Z1Const<T, (MS > 0 ? MS : 1)> kc(c);
    const double *tab = TAB ? g.tab64 + off : nullptr;
    cx<T> acc[NO][5];
    if constexpr (MS == 0) {
        // species by species, every node's input of a species in flight together
#pragma unroll
        for (int i = 0; i < NO; ++i)
#pragma unroll
            for (int m = 0; m < 5; ++m) acc[i][m] = mk<T>(T(0), T(0));
        for (int jsp = 0; jsp < S; ++jsp) {
            const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specA) + (long long)jsp * NC + off;
            cx<T> uin[NO];
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                int p, e;
                const bool ok = F::template in_pos<1>(i, p, e) && p < Pact;
                uin[i] = ok ? ct::gld(src + e * rs + p) : mk<T>(T(0), T(0));
            }
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                int p, e;
                const bool ok = F::template in_pos<1>(i, p, e) && p < Pact;
                z1_species<T>(c, kw, tab, NC, S, jsp, e, ok, ok ? e * rs + p : 0, uin[i], acc[i]);
            }
        }
    } else {
        Poisson<T> pd;
        if constexpr (!TAB) pd = Poisson<T>(g, c, zt.x, zt.y);
        static_for<NO>([&](auto I) __attribute__((always_inline)) {
            constexpr int i = I;
            int p, e;
            const bool ok = F::template in_pos<1>(i, p, e) && p < Pact;
            const long long ti = ok ? e * rs + p : 0;
            cx<T> *src = reinterpret_cast<cx<T> *>(a.specA) + off + ti;
            cx<T> u[MS];
#pragma unroll
            for (int j = 0; j < MS; ++j) u[j] = (ok && j < S) ? ct::gld(src + (long long)j * NC) : mk<T>(T(0), T(0));
            z1_node<T, MS>(kc, a.diff != 0, kw, pd, tab, NC, S, es, e, ok, ti, u, acc[i], src);
        });
    }
    int ph = 0;
    z1_inverse<T, F, NO>(g, a, kw, lds, ph, tw, Pact, rs, off, acc);
}

// Z2: forward z transform of the ten dPhi/dn spectra, back-convolution with conj(w_hat)
// (eq. muHS; the vector parts enter as +i k_d times a w3 weight), plus the electrostatic
// spectra Z1 left in specA, times 1/N, inverse z -> specA.  Z2_POISSON instead forms the
// potential of weighted source spectra, Z2_BALL the ball averages of the RFD screening operator.
// Weights: tables in FP64, on the fly in FP32.
template <typename T, int L, int P, int NTB>
__global__ __launch_bounds__(NTB) void k_z2c(Geo g_in, Z2Args a) {
    using F = ct::Fft<T, typename ct::PlanT<T, L>::type, P, NTB, false, 2>;
    constexpr int NO = F::template nout<-1>();
    static_assert(NO == F::template nin<1>(), "inverse must start where the forward ends");
    constexpr bool TAB = std::is_same<T, double>::value;
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    __shared__ cx<T> lds[F::LDS_ELEMS];
    const Consts &c = *g.cs;
    const int Kx = g.Kx, S = g.S;
    const long long NC = g.NC;
    static_assert(NTB % P == 0, "a thread keeps one column");
    const ZTile zt = z_tile<P>(g);
    const int Pact = zt.Pact;
    const long long rs = (long long)g.ny * Kx;
    const long long off = zt.off;
    const cx<T> *tw = twp<T>(g, 2);
    const ZWave<T> kw(c, zt.x, zt.y);
    // position of output register i of the forward transforms (recomputed at each use: a few
    // instructions from the thread index instead of registers held through the kernel)
    auto ee = [&](int i) {
        int p, e;
        F::template out_pos<-1>(i, p, e);
        return e;
    };
    auto okk = [&](int i) {
        int p, e;
        return F::template out_pos<-1>(i, p, e) && p < Pact;
    };
    auto ti = [&](int i) {
        int p, e;
        const bool ok = F::template out_pos<-1>(i, p, e) && p < Pact;
        return ok ? e * rs + p : 0;
    };
    cx<T> v[F::V];
    int ph = 0;
    // FP32: the forward twiddles in registers, shared by the input transforms (in FP64 the
    // register budget is better spent on the transforms themselves)
    constexpr bool TWR = std::is_same<T, float>::value;
    typename F::template TwReg<-1> trf;
    if constexpr (TWR) F::template load_tw<-1>(trf, tw);
    auto fwd = [&]() {
        if constexpr (TWR) F::template run<-1>(v, lds, ph, trf);
        else F::template run<-1>(v, lds, ph, tw);
    };
    auto load_fwd = [&](const cx<T> *src) {
#pragma unroll
        for (int i = 0; i < F::template nin<-1>(); ++i) {
            int p, e;
            const bool ok = F::template in_pos<-1>(i, p, e);
            v[i] = (ok && p < Pact) ? ct::gld(src + e * rs + p) : mk<T>(T(0), T(0));
        }
        fwd();
    };
    auto inv_store = [&](cx<T> *dst) {
        F::template run<1>(v, lds, ph, tw);
#pragma unroll
        for (int i = 0; i < F::template nout<1>(); ++i) {
            int p, e;
            const bool ok = F::template out_pos<1>(i, p, e);
            if (ok && p < Pact) ct::gst(dst + e * rs + p, v[i]);
        }
    };

    if (a.mode == Z2_BALL) {
        // ball average of every source field (the RFD screening operator at one radius):
        // specA[i] x B(|k| radius) / N -> specB[i]
        double m[NO];
#pragma unroll
        for (int i = 0; i < NO; ++i) m[i] = ball_mean<double>((double)kw.kmag(ee(i)), a.radius) * c.invN;
        for (int is = 0; is < a.nsrc; ++is) {
            load_fwd(reinterpret_cast<const cx<T> *>(a.specA) + (long long)is * NC + off);
#pragma unroll
            for (int i = 0; i < NO; ++i) v[i] = mk<T>(T((double)v[i].x * m[i]), T((double)v[i].y * m[i]));
            inv_store(reinterpret_cast<cx<T> *>(a.specB) + (long long)is * NC + off);
        }
        return;
    }
    if (a.mode == Z2_POISSON) {
        // phi_hat = 4 pi l_B (sum_j w_j src_j) / D(k), zero mode 0; x invN; output in specA[0].
        double acc[NO][2];
#pragma unroll
        for (int i = 0; i < NO; ++i) acc[i][0] = acc[i][1] = 0.0;
        for (int is = 0; is < a.nsrc; ++is) {
            load_fwd(reinterpret_cast<const cx<T> *>(a.specA) + (long long)is * NC + off);
            double wj = 0.0;   // a.wsrc[is] read with constant indices (no scratch copy of the arguments)
#pragma unroll
            for (int k = 0; k < DFT_MAX_SPECIES; ++k)
                if (k == is) wj = a.wsrc[k];
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                acc[i][0] += wj * (double)v[i].x;
                acc[i][1] += wj * (double)v[i].y;
            }
        }
        const Poisson<double> pd(g, c, zt.x, zt.y);
#pragma unroll
        for (int i = 0; i < NO; ++i) {
            double m = 0.0;
            if (!kw.zero(ee(i))) m = c.four_pi_lB / pd.denom(ee(i)) * c.invN;
            v[i] = mk<T>(T(acc[i][0] * m), T(acc[i][1] * m));
        }
        inv_store(reinterpret_cast<cx<T> *>(a.specA) + off);
        return;
    }

    // six sums of the derivative spectra: u0..u3 and v1 = sum_d i k_d dPhi_V1,d, v2 likewise
    cx<T> u[6][NO];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int i = 0; i < NO; ++i) u[m][i] = mk<T>(T(0), T(0));
    // Eight forward transforms: along a z pencil k_x and k_y are constant, so the x and y parts of
    // each vector sum, i k_x dPhi_x + i k_y dPhi_y, are combined before one transform; the z parts
    // are transformed and multiplied by i k_z after.  Transform t: 0..3 the scalars (u0..u3);
    // 4, 6 the combined x, y parts of V1, V2; 5, 7 their z parts.
    // compact layout: slots 4 and 7 already hold i k_x dPhi_x + i k_y dPhi_y and all eight inputs
    // are plain spectra; in FP32 tiles of at most eight values per thread each is fetched while the
    // previous one transforms (FP64 tiles have no registers to spare for it)
    constexpr bool PF = std::is_same<T, float>::value && NO <= 8;
    constexpr int NIN = F::template nin<-1>();
    cx<T> vin[NIN];
    auto slot_of = [](int t) { return t < 4 ? t : (t == 4 ? 4 : (t == 5 ? 6 : (t == 6 ? 7 : 9))); };
    auto fetch = [&](int t) {
        const int al = slot_of(t);
        const cx<T> *src = reinterpret_cast<const cx<T> *>(a.specB) + (long long)al * NC + off;
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            int p, e;
            const bool ok = F::template in_pos<-1>(i, p, e);
            vin[i] = (ok && p < Pact) ? ct::gld(src + e * rs + p) : mk<T>(T(0), T(0));
        }
    };
    if (PF && g.compact) fetch(0);
    for (int t = 0; t < 8; ++t) {
        const int m = t < 4 ? t : (t < 6 ? 4 : 5);
        if (g.compact) {
            if constexpr (PF) {
#pragma unroll
                for (int i = 0; i < NIN; ++i) v[i] = vin[i];
                if (t + 1 < 8) fetch(t + 1);
                fwd();
            } else {
                load_fwd(reinterpret_cast<const cx<T> *>(a.specB) + (long long)slot_of(t) * NC + off);
            }
        } else if (t < 4 || t == 5 || t == 7) {
            const int al = t < 4 ? t : (t == 5 ? 6 : 9);
            load_fwd(reinterpret_cast<const cx<T> *>(a.specB) + (long long)al * NC + off);
        } else {
            const int al = t == 4 ? 4 : 7;
            const cx<T> *sx = reinterpret_cast<const cx<T> *>(a.specB) + (long long)al * NC + off;
            const cx<T> *sy = sx + NC;
#pragma unroll
            for (int i = 0; i < F::template nin<-1>(); ++i) {
                int p, e;
                const bool ok = F::template in_pos<-1>(i, p, e) && p < Pact;
                cx<T> w = mk<T>(T(0), T(0));
                if (ok) {
                    const cx<T> fx = ct::gld(sx + e * rs + p), fy = ct::gld(sy + e * rs + p);
                    const T kx = kw.comp(e, 0), ky = kw.comp(e, 1);
                    w = mk<T>(-(kx * fx.y + ky * fy.y), kx * fx.x + ky * fy.x);   // i k_x fx + i k_y fy
                }
                v[i] = w;
            }
            fwd();
        }
#pragma unroll
        for (int i = 0; i < NO; ++i) {
            cx<T> w = v[i];
            if (t == 5 || t == 7) {
                const T kd = kw.comp(ee(i), 2);
                w = mk<T>(-kd * w.y, kd * w.x);   // + i k_z w
            }
#pragma unroll
            for (int mm = 0; mm < 6; ++mm)
                if (mm == m) { u[mm][i].x += w.x; u[mm][i].y += w.y; }
        }
    }
    const T invN = T(c.invN);
    constexpr int NOF = TAB ? 1 : NO;
    T kmag[NOF];
    if constexpr (!TAB) {
#pragma unroll
        for (int i = 0; i < NO; ++i) kmag[i] = kw.kmag(ee(i));
    }
    // FP32: the electrostatic spectra of species is + 1 fetched while species is transforms
    // (slot is + 1 is written only in the next iteration, after every read of it)
    cx<T> evn[NO];
    const bool es = c.es != 0;   // read once (a read after the stores below would be repeated)
    auto fetch_es = [&](int is) {
        const cx<T> *esrc = reinterpret_cast<const cx<T> *>(a.specA) + (long long)is * NC + off;
#pragma unroll
        for (int i = 0; i < NO; ++i) evn[i] = (es && okk(i)) ? ct::gld(esrc + ti(i)) : mk<T>(T(0), T(0));
    };
    if constexpr (PF) fetch_es(0);
    for (int is = 0; is < S; ++is) {
        const T Ri = T(c.R[is]), a0 = T(c.i4piR2[is]), a1 = T(c.i4piR[is]);
        if constexpr (!PF) fetch_es(is);
        cx<T> ev[NO];
#pragma unroll
        for (int i = 0; i < NO; ++i) ev[i] = evn[i];
        if (PF && is + 1 < S) fetch_es(is + 1);
#pragma unroll
        for (int i = 0; i < NO; ++i) {
            T w2, w3;
            if constexpr (TAB) {
                const double *tab = g.tab64 + off;
                w2 = ct::cld(tab + (long long)is * NC + ti(i));
                w3 = ct::cld(tab + (long long)(S + is) * NC + ti(i));
            } else {
                weight_w2_w3<T>(kmag[i], Ri, w2, w3);
            }
            const T s2x = u[0][i].x * a0 + u[1][i].x * a1 + u[2][i].x;
            const T s2y = u[0][i].y * a0 + u[1][i].y * a1 + u[2][i].y;
            const T s3x = u[3][i].x + u[4][i].x * a1 + u[5][i].x;
            const T s3y = u[3][i].y + u[4][i].y * a1 + u[5][i].y;
            T ex = -(s2x * w2 + s3x * w3);
            T ey = -(s2y * w2 + s3y * w3);
            ex += ev[i].x;
            ey += ev[i].y;
            v[i] = mk<T>(ex * invN, ey * invN);
        }
        inv_store(reinterpret_cast<cx<T> *>(a.specA) + (long long)is * NC + off);
    }
}

// ------------------------------------------------------------------ x passes
// Two real rows (r0, r0 + 1) travel as the real and imaginary parts of one complex row:
// the forward transform C of c = a + i b gives A_k = (C_k + conj C_{L-k}) / 2 and
// B_k = (C_k - conj C_{L-k}) / (2i); the inverse rebuilds C from the Hermitian halves.
// A tile holds PB such row pairs; the block has PB L / 4 threads, and with the x schedules
// (radices <= 4, forward starting with 4) each thread ends an inverse transform holding
// the same four columns of its pencil for every field, so the nodewise work of X2 runs on
// registers.
template <int L>
struct XTile {
    static constexpr int PB = (L % 3 == 0) ? 768 / L : 1024 / L;
    static constexpr int NTB = PB * L / 4;
    static constexpr int KX = L / 2 + 1;
    static constexpr int PAD = 0;
};

// Element e of the full spectrum of a real row from its half spectrum (Hermitian).
template <typename T, int L>
__device__ __forceinline__ cx<T> half_at(const cx<T> *row, int e) {
    constexpr int KX = L / 2 + 1;
    cx<T> v;
    if (e < KX) {
        v = ct::gld(row + e);
        if (e == 0 || 2 * e == L) v.y = T(0);
    } else {
        v = conjg(ct::gld(row + (L - e)));
    }
    return v;
}

// Value v of lane src of the wave (cross-lane permute, 32 bits at a time; no memory access).
template <typename T>
__device__ __forceinline__ cx<T> lane_value(cx<T> v, int src) {
    constexpr int W = (int)(sizeof(cx<T>) / 4);
    int w[W];
    __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = __builtin_amdgcn_ds_bpermute(src << 2, w[k]);
    cx<T> r;
    __builtin_memcpy(&r, w, sizeof(r));
    return r;
}

// Inputs of an inverse x transform: for the row pair of register i, C_e = A_e + i B_e from the
// half spectra of rows r0 and r0 + 1 (B = 0 past the last row; pairs past Pact read as zero).
// In a wave-private tile lane b of a pencil holds e = b + q L/4 (q = 0..3); the elements
// e > L/2 are conj(A_{L-e}), and L - e is an element that lane (L/4 - b) mod L/4 of the same
// pencil loads for q = 0 or 1, so they come by cross-lane permutes instead of second loads.
// Paired x tiles (k_x2p): two waves share each row pair, so the pencil slot p of a wave-private
// tile (ppw = 256 / L slots per wave) maps to row pair (p / (2 ppw)) ppw + p % ppw of the block.
template <int L>
__device__ __forceinline__ int paired_pair(int p) {
    constexpr int ppw = 256 / L;
    return (p / (2 * ppw)) * ppw + p % ppw;
}

template <typename T, int L, class F, bool PAIRED = false>
__device__ __forceinline__ void load_row_pairs(const cx<T> *in, long long pair0, int Pact, long long rows, cx<T> *c) {
    constexpr int KX = L / 2 + 1;
    if constexpr (F::WP) {
        constexpr int Q = L / 4;
        static_assert(F::template nin<1>() == 4, "one radix-4 butterfly per thread");
        int p, b;
        F::template in_pos<1>(0, p, b);
        if constexpr (PAIRED) p = paired_pair<L>(p);
        const bool ok = p < Pact;
        const long long r0 = 2 * (pair0 + p);
        const bool okb = ok && r0 + 1 < rows;
        const cx<T> *ra = in + r0 * KX, *rb = ra + KX;
        const cx<T> z = mk<T>(T(0), T(0));
        cx<T> A0 = z, A1 = z, An = z, B0 = z, B1 = z, Bn = z;
        if (ok) {
            A0 = ct::gld(ra + b);
            A1 = ct::gld(ra + Q + b);
            if (b == 0) {
                A0.y = T(0);
                An = ct::gld(ra + 2 * Q);   // the Nyquist element
                An.y = T(0);
            }
        }
        if (okb) {
            B0 = ct::gld(rb + b);
            B1 = ct::gld(rb + Q + b);
            if (b == 0) {
                B0.y = T(0);
                Bn = ct::gld(rb + 2 * Q);
                Bn.y = T(0);
            }
        }
        const int lane = (int)(threadIdx.x & 63);
        const int src = lane - b + ((Q - b) & (Q - 1));
        const cx<T> a1 = lane_value(A1, src), a0 = lane_value(A0, src);
        const cx<T> b1 = lane_value(B1, src), b0 = lane_value(B0, src);
        const cx<T> A2 = b == 0 ? An : conjg(a1), A3 = b == 0 ? conjg(a1) : conjg(a0);
        const cx<T> B2 = b == 0 ? Bn : conjg(b1), B3 = b == 0 ? conjg(b1) : conjg(b0);
        c[0] = mk<T>(A0.x - B0.y, A0.y + B0.x);
        c[1] = mk<T>(A1.x - B1.y, A1.y + B1.x);
        c[2] = mk<T>(A2.x - B2.y, A2.y + B2.x);
        c[3] = mk<T>(A3.x - B3.y, A3.y + B3.x);
    } else {
        static_assert(!PAIRED, "paired tiles are wave-private");
#pragma unroll
        for (int i = 0; i < F::template nin<1>(); ++i) {
            int p, e;
            const bool ok = F::template in_pos<1>(i, p, e) && p < Pact;
            cx<T> cv = mk<T>(T(0), T(0));
            if (ok) {
                const long long r0 = 2 * (pair0 + p);
                const cx<T> A = half_at<T, L>(in + r0 * KX, e);
                cx<T> B = mk<T>(T(0), T(0));
                if (r0 + 1 < rows) B = half_at<T, L>(in + (r0 + 1) * KX, e);
                cv = mk<T>(A.x - B.y, A.y + B.x);
            }
            c[i] = cv;
        }
    }
}

// Half spectra of the two real rows of every row pair from the forward transform of the pair
// (C held in split): A_k = (C_k + conj C_{L-k}) / 2, B_k = (C_k - conj C_{L-k}) / (2i).  In a
// wave-private tile each wave splits its own pencils (lanes along k); otherwise the block does
// (split must have been synchronized accordingly by the caller).
// With dkx > 0 both half spectra are multiplied by i k_x (k_x = k dkx, zero on the Nyquist column).
template <typename T, int L, class F, bool PAIRED = false>
__device__ __forceinline__ void split_rows(const cx<T> *split, cx<T> *out, long long pair0, int Pact, long long rows,
                                           T dkx = T(0)) {
    constexpr int KX = L / 2 + 1;
    auto coeffs = [&](int p, int k, cx<T> &A, cx<T> &B) {
        const cx<T> ck = split[F::lidx(p, k)];
        const cx<T> cm = split[F::lidx(p, k == 0 ? 0 : L - k)];
        A = mk<T>(T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y - cm.y));
        B = mk<T>(T(0.5) * (ck.y + cm.y), T(-0.5) * (ck.x - cm.x));
        if (dkx > T(0)) {
            const T kx = (L % 2 == 0 && 2 * k == L) ? T(0) : T(k) * dkx;
            A = mk<T>(-kx * A.y, kx * A.x);
            B = mk<T>(-kx * B.y, kx * B.x);
        }
    };
    auto one = [&](int p, int pr, int k) {
        cx<T> A, B;
        coeffs(p, k, A, B);
        const long long r0 = 2 * (pair0 + pr);
        ct::gst(out + r0 * KX + k, A);
        if (r0 + 1 < rows) ct::gst(out + (r0 + 1) * KX + k, B);
    };
    if constexpr (F::WP) {
        // lane b of a pencil writes k = b and b + L/4 of both rows; the Nyquist element k = L/2
        // goes to row r0 from lane 0 and to row r0 + 1 from lane 1 (one store instead of two)
        constexpr int nb = L / 4;
        const int lane = (int)threadIdx.x % 64;
        const int p = ((int)threadIdx.x / 64) * (64 / nb) + lane / nb;
        const int pr = PAIRED ? paired_pair<L>(p) : p;
        const int b = lane % nb;
        if (pr < Pact) {
            one(p, pr, b);
            one(p, pr, b + nb);
            if (b < 2) {
                cx<T> A, B;
                coeffs(p, 2 * nb, A, B);
                const long long r = 2 * (pair0 + pr) + b;
                if (r < rows) ct::gst(out + r * KX + 2 * nb, b == 0 ? A : B);
            }
        }
    } else {
        static_assert(!PAIRED, "paired tiles are wave-private");
        for (int j = threadIdx.x; j < Pact * KX; j += (int)blockDim.x) {
            const int p = j / KX;
            one(p, p, j - p * KX);
        }
    }
}

// Nodewise variants of X2: FP64 eq. (Phi); FP32 differences from the reference (eq. (Phi),
// x2_node_diff); FP64 with an alternative functional chosen by X2Args::hs.
enum X2Node { X2N_FP64 = 0, X2N_D32 = 1, X2N_ALT = 2 };

// X2: ten weighted-density spectra after the y inverse -> inverse x -> pointwise dPhi/dn
// (eq. Phi) -> forward x -> half spectra, in place in specB.  Register budget of two waves per
// SIMD: the FP64 kernel would otherwise take one (344 registers; a few spills are cheaper).
template <typename T, int L, int NODE = X2N_FP64>
__global__ __launch_bounds__(XTile<L>::NTB) __attribute__((amdgpu_waves_per_eu(2))) void
k_x2c(Geo g_in, X2Args a) {
    using XT = XTile<L>;
    constexpr int PB = XT::PB, NTB = XT::NTB, KX = XT::KX;
    using F = ct::Fft<T, typename ct::XPlan<L>::type, PB, NTB, true, 2, XT::PAD>;
    constexpr int NO = F::template nout<1>();
    static_assert(NO == F::template nin<-1>(), "forward must start where the inverse ends");
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    const T dk0 = T(g.cs->dk[0]);   // k_x step, read before any store
    __shared__ cx<T> lds[F::LDS_ELEMS + F::TILE];
    cx<T> *split = lds + F::LDS_ELEMS;
    const long long N = g.N, NC = g.NC;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * PB;
    const int Pact = (int)min((long long)PB, npairs - pair0);
    const cx<T> *tw = twp<T>(g, 0);
    // wave-private tiles: the twiddles of all 20 transforms, once, in registers
    typename F::Twiddles trw;
    if constexpr (F::WP) F::load_twiddles(trw, tw);
    const bool n3only = a.mode == X2_N3_ONLY;
    const int nf = n3only ? 1 : DFT_NALPHA;
    // X2N_D32 (FP32 differences from the reference, no FP64 copies asked for): the nodewise
    // difference in FP32 (x2_node_diff); the launcher picks it.
    constexpr bool D32 = NODE == X2N_D32;
    static_assert(!D32 || std::is_same<T, float>::value, "FP32 difference path");
    cx<T> vals[DFT_NALPHA][NO];
    cx<T> v[F::V];
    int ph = 0;
    // all loads first (every field's inputs in flight together), then the transforms
    static_assert(NO == F::template nin<1>(), "inputs and outputs share registers");
#pragma unroll
    for (int f = 0; f < DFT_NALPHA; ++f) {
        if (f >= nf) continue;
        if (f == 7 && g.compact) {
            // compact layout: n_V2,x = -i k_x n3 (k_x zero on the Nyquist column), formed here
            const T dkx = T(g.cs->dk[0]);
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                int p, e;
                F::template in_pos<1>(i, p, e);
                const T kx = (L % 2 == 0 && 2 * e == L) ? T(0) : T(e <= L / 2 ? e : e - L) * dkx;
                vals[7][i] = mk<T>(kx * vals[3][i].y, -kx * vals[3][i].x);
            }
            continue;
        }
        load_row_pairs<T, L, F>(reinterpret_cast<const cx<T> *>(a.specB) + (long long)f * NC, pair0, Pact, rows,
                                vals[f]);
    }
    // D32: the reference weighted densities of a register's two nodes, fetched one register
    // ahead of the nodewise work (the first before the transforms) so their latency is hidden
    constexpr int NRB = D32 ? 2 : 1;
    float nrc[NRB][2][DFT_NALPHA];
    auto fetch_nref = [&](int i, float (&dst)[2][DFT_NALPHA]) {
        int p, e;
        const bool ok = F::template out_pos<1>(i, p, e) && p < Pact;
        const long long r0 = 2 * (pair0 + p);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool okh = ok && r0 + h < rows;
            const long long idx = (r0 + h) * L + e;
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) dst[h][f] = okh ? ct::cld(a.nref + f * N + idx) : 0.0f;
        }
    };
    if constexpr (D32) fetch_nref(0, nrc[0]);
#pragma unroll
    for (int f = 0; f < DFT_NALPHA; ++f) {
        if (f >= nf) continue;
#pragma unroll
        for (int i = 0; i < NO; ++i) v[i] = vals[f][i];
        if constexpr (F::WP) F::template run<1>(v, lds, ph, trw);
        else F::template run<1>(v, lds, ph, tw);
#pragma unroll
        for (int i = 0; i < NO; ++i) vals[f][i] = v[i];
    }
    double mloc = -INFINITY;
    int flag = 0;
#pragma unroll
    for (int i = 0; i < NO; ++i) {
        if constexpr (D32) {
            if (i + 1 < NO) fetch_nref(i + 1, nrc[(i + 1) % NRB]);
        }
        int p, e;
        if (!(F::template out_pos<1>(i, p, e) && p < Pact)) continue;
        const long long r0 = 2 * (pair0 + p);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long r = r0 + h;
            if (r >= rows) break;
            const long long idx = r * L + e;
            if (n3only) {
                double n3 = h == 0 ? (double)vals[0][i].x : (double)vals[0][i].y;
                if (a.nref) n3 += (double)a.nref[3 * N + idx];
                if (!isfinite(n3)) flag |= 5;   // 1: evaluation non-finite, 4: n3 non-finite
                mloc = fmax(mloc, n3);
                continue;
            }
            if constexpr (D32) {
                float dn[DFT_NALPHA], dd[DFT_NALPHA];
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) dn[f] = h == 0 ? vals[f][i].x : vals[f][i].y;
                x2_node_diff(nrc[i % NRB][h], dn, dd, mloc, flag);
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) {
                    if (h == 0) vals[f][i].x = dd[f];
                    else vals[f][i].y = dd[f];
                }
            } else {
                double n[DFT_NALPHA], d[DFT_NALPHA];
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) n[f] = h == 0 ? (double)vals[f][i].x : (double)vals[f][i].y;
                x2_node<NODE == X2N_ALT>(a, N, idx, n, d, mloc, flag);
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) {
                    if (h == 0) vals[f][i].x = T(d[f]);
                    else vals[f][i].y = T(d[f]);
                }
            }
        }
        if (!n3only && r0 + 1 >= rows) {
            // the missing partner row transforms as zero
#pragma unroll
            for (int f = 0; f < DFT_NALPHA; ++f) vals[f][i].y = T(0);
        }
    }
    if (flag & 4) mloc = INFINITY;   // the n3 bound needs finite n3 only
    block_reduce_nt<true, NTB>(mloc, flag, a.red.mpart + blockIdx.x, a.red.mflag + blockIdx.x);
    if (n3only) return;
#pragma unroll
    for (int f = 0; f < DFT_NALPHA; ++f) {
#pragma unroll
        for (int i = 0; i < NO; ++i) v[i] = vals[f][i];
        if constexpr (F::WP) F::template run<-1>(v, lds, ph, trw);
        else F::template run<-1>(v, lds, ph, tw);
#pragma unroll
        for (int i = 0; i < F::template nout<-1>(); ++i) {
            int p, e;
            if (F::template out_pos<-1>(i, p, e)) split[F::lidx(p, e)] = v[i];
        }
        F::sync();
        // compact layout: the x components of the vector derivatives leave multiplied by i k_x
        const T dkx = (g.compact && (f == 4 || f == 7)) ? dk0 : T(0);
        split_rows<T, L, F>(split, reinterpret_cast<cx<T> *>(a.specB) + (long long)f * NC, pair0, Pact, rows, dkx);
    }
}

// X2 on wave-private tiles with the ten fields of every row pair shared by two waves of the
// block.  Wave h of a pair transforms five fields, x2_half_field(h, 0..4) (h = 0: n0..n3 and
// nV2,x, so the compact layout forms nV2,x = -i k_x n3 in the same wave; h = 1: the nV1
// components and nV2,y, nV2,z), and does the nodewise work at the nodes of its registers
// q = 2h, 2h + 1; the other five values of those nodes come from the partner wave through LDS,
// and their derivatives go back the same way.  Half the fields per wave halves the registers the
// transforms hold (FP32: three waves fit per SIMD where k_x2c fits two; FP64: two without the
// spills of k_x2c), for the same arithmetic in the same order.  Nodewise work: FP32, the
// difference from the reference (x2_node_diff, FP32-mixed evaluations); FP64, x2_node with
// eq. (Phi), every mode but the n3-only one.
template <typename T, int L>
struct XPairTile {
    static constexpr int PF = 1024 / L;   // pencil slots of a block (four waves)
    static constexpr int NTB = 256;
    static constexpr int PB = PF / 2;     // row pairs of a block
    static constexpr int WPE = sizeof(T) == 4 ? 3 : 2;   // waves per SIMD the registers allow
};

__host__ __device__ constexpr int x2_half_field(int h, int j) {
    return h == 0 ? (j < 4 ? j : 7) : (j < 3 ? 4 + j : 5 + j);
}

// Exchange slot s (0..639: field j, register k, lane as (2 j + k) 64 + lane) of wave w in the
// wave's own LDS regions of the transform tile: pencils w 256/L.. of the two transform buffers
// and of the split buffer, 256 elements each (whole pencils of a wave-private tile).
template <class F, typename T>
__device__ __forceinline__ cx<T> *x2p_slot(cx<T> *lds, int w, int s) {
    static_assert(F::TILE == 1024 && F::LDS_ELEMS == 2 * F::TILE, "four waves of 256 elements per buffer");
    return lds + (s >> 8) * F::TILE + w * 256 + (s & 255);
}

// Nodewise work of one paired wave (H: its half) with the swap through LDS: the own fields at the
// partner's registers go out to the own slots; after a barrier the wave takes the partner's fields
// at its own registers q = 2H + k from the partner's slots, one register at a time, and leaves the
// partner's derivatives in the same place; after a second barrier it reads its own derivatives at
// the partner's registers back.  Between the barriers only the partner touches a wave's slots;
// outside them the slots are the wave's own transform regions.  Every wave of the block passes
// both barriers.
template <typename T, int L, class F, int H>
__device__ __forceinline__ void x2p_swap_and_nodes(const X2Args &a, long long N, long long pair0, int Pact,
                                                   long long rows, cx<T> *lds, int wave, int lane,
                                                   cx<T> (&vals)[5][4], double &mloc, int &flag) {
    constexpr int QP = 2 * (1 - H);   // the partner's registers
    F::sync();   // the forward transforms' reads of the same regions precede the writes below
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) *x2p_slot<F>(lds, wave, (2 * j + k) * 64 + lane) = vals[j][QP + k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = 2 * H + k;
        int p, e;
        F::template out_pos<1>(i, p, e);
        const int pr = paired_pair<L>(p);
        const long long r0 = 2 * (pair0 + pr);
        cx<T> oth[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) oth[j] = *x2p_slot<F>(lds, wave ^ 1, (2 * j + k) * 64 + lane);
#pragma unroll
        for (int hr = 0; hr < 2; ++hr) {
            const bool ok = pr < Pact && r0 + hr < rows;
            const long long idx = (r0 + hr) * L + e;
            T dn[DFT_NALPHA], dd[DFT_NALPHA];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                dn[x2_half_field(H, j)] = hr == 0 ? vals[j][i].x : vals[j][i].y;
                dn[x2_half_field(1 - H, j)] = hr == 0 ? oth[j].x : oth[j].y;
            }
            if (ok) {
                if constexpr (sizeof(T) == 4) {
                    float nr[DFT_NALPHA];
#pragma unroll
                    for (int f = 0; f < DFT_NALPHA; ++f) nr[f] = ct::cld(a.nref + f * N + idx);
                    x2_node_diff(nr, dn, dd, mloc, flag);
                } else {
                    x2_node<false>(a, N, idx, dn, dd, mloc, flag);
                }
            } else {
#pragma unroll
                for (int f = 0; f < DFT_NALPHA; ++f) dd[f] = T(0);   // pairs past Pact, the missing partner row
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                if (hr == 0) {
                    vals[j][i].x = dd[x2_half_field(H, j)];
                    oth[j].x = dd[x2_half_field(1 - H, j)];
                } else {
                    vals[j][i].y = dd[x2_half_field(H, j)];
                    oth[j].y = dd[x2_half_field(1 - H, j)];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) *x2p_slot<F>(lds, wave ^ 1, (2 * j + k) * 64 + lane) = oth[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) vals[j][QP + k] = *x2p_slot<F>(lds, wave, (2 * j + k) * 64 + lane);
    F::sync();   // the reads above precede the inverse transforms' writes to the same regions
}

template <typename T, int L>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(XPairTile<T, L>::WPE))) void
k_x2p(Geo g_in, X2Args a) {
    using XP = XPairTile<T, L>;
    constexpr int PF = XP::PF, NTB = XP::NTB, PB = XP::PB;
    using F = ct::Fft<T, typename ct::XPlan<L>::type, PF, NTB, true, 2, 0>;
    static_assert(F::WP, "paired tiles are wave-private");
    static_assert(NTB == 256, "the launch bound above");
    static_assert(F::template nout<1>() == 4 && F::template nin<-1>() == 4, "one radix-4 butterfly per thread");
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    const T dk0 = T(g.cs->dk[0]);   // k_x step, read before any store
    __shared__ cx<T> lds[F::LDS_ELEMS + F::TILE];
    cx<T> *split = lds + F::LDS_ELEMS;
    const long long N = g.N, NC = g.NC;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * PB;
    const int Pact = (int)min((long long)PB, npairs - pair0);
    const cx<T> *tw = twp<T>(g, 0);
    typename F::Twiddles trw;
    F::load_twiddles(trw, tw);
    const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64, h = wave & 1;
    cx<T> vals[5][4];
    cx<T> v[F::V];
    int ph = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int f = x2_half_field(h, j);
        if (f == 7 && g.compact) {
            // compact layout: n_V2,x = -i k_x n3 (k_x zero on the Nyquist column), from field 3 (j = 3)
            const T dkx = T(g.cs->dk[0]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int p, e;
                F::template in_pos<1>(i, p, e);
                const T kx = (L % 2 == 0 && 2 * e == L) ? T(0) : T(e <= L / 2 ? e : e - L) * dkx;
                vals[j][i] = mk<T>(kx * vals[3][i].y, -kx * vals[3][i].x);
            }
            continue;
        }
        load_row_pairs<T, L, F, true>(reinterpret_cast<const cx<T> *>(a.specB) + (long long)f * NC, pair0, Pact, rows,
                                      vals[j]);
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = vals[j][i];
        F::template run<1>(v, lds, ph, trw);
#pragma unroll
        for (int i = 0; i < 4; ++i) vals[j][i] = v[i];
    }
    double mloc = -INFINITY;
    int flag = 0;
    // the halves take constant register indices (a run-time choice would put vals in scratch)
    if (h == 0) x2p_swap_and_nodes<T, L, F, 0>(a, N, pair0, Pact, rows, lds, wave, lane, vals, mloc, flag);
    else x2p_swap_and_nodes<T, L, F, 1>(a, N, pair0, Pact, rows, lds, wave, lane, vals, mloc, flag);
    if (flag & 4) mloc = INFINITY;   // the n3 bound needs finite n3 only
    block_reduce_nt<true, NTB>(mloc, flag, a.red.mpart + blockIdx.x, a.red.mflag + blockIdx.x);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = vals[j][i];
        F::template run<-1>(v, lds, ph, trw);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int p, e;
            if (F::template out_pos<-1>(i, p, e)) split[F::lidx(p, e)] = v[i];
        }
        F::sync();
        const int f = x2_half_field(h, j);
        const T dkx = (g.compact && (f == 4 || f == 7)) ? dk0 : T(0);
        split_rows<T, L, F, true>(split, reinterpret_cast<cx<T> *>(a.specB) + (long long)f * NC, pair0, Pact, rows, dkx);
    }
}

// X1: real rows of field blockIdx.y (plain, or the line-search trial point
// rho0 + alpha (g0 - rho0), written out; FP32-mixed: minus the reference) -> forward x ->
// half spectra.
template <typename T, int L>
__global__ __launch_bounds__(XTile<L>::NTB) void k_x1c(Geo g_in, XFwdArgs a) {
    using XT = XTile<L>;
    constexpr int PB = XT::PB, NTB = XT::NTB, KX = XT::KX;
    using F = ct::Fft<T, typename ct::XPlan<L>::type, PB, NTB, true, 2, XT::PAD>;
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    resolve_roles(a);
    // wave-private tiles: twiddles fetched up front, with the data
    typename F::Twiddles trw;
    if constexpr (F::WP) F::load_twiddles(trw, twp<T>(g_in, 0));
    __shared__ cx<T> lds[F::LDS_ELEMS + F::TILE];
    cx<T> *split = lds + F::LDS_ELEMS;
    const int f = blockIdx.y;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * PB;
    const int Pact = (int)min((long long)PB, npairs - pair0);
    const long long foff = (long long)f * g.N;
    const bool trial = a.mode == XF_TRIAL;
    const double alpha = trial ? *a.alpha : 0.0;
    cx<T> v[F::V];
#pragma unroll
    for (int i = 0; i < F::template nin<-1>(); ++i) {
        int p, e;
        const bool ok = F::template in_pos<-1>(i, p, e) && p < Pact;
        double x[2] = {0.0, 0.0};
        if (ok) {
            const long long r0 = 2 * (pair0 + p);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const long long r = r0 + h;
                if (r >= rows) break;
                const long long idx = foff + r * L + e;
                double xv;
                if (trial) {
                    const double r0v = ct::cld(a.src + idx);
                    xv = fma(alpha, ct::cld(a.g0 + idx) - r0v, r0v);
                    if (a.rho_t) ct::gst(a.rho_t + idx, xv);
                } else {
                    xv = ct::cld(a.src + idx);
                }
                if (a.ref) xv -= ct::cld(a.ref + idx);
                x[h] = xv;
            }
        }
        v[i] = mk<T>(T(x[0]), T(x[1]));
    }
    int ph = 0;
    if constexpr (F::WP) F::template run<-1>(v, lds, ph, trw);
    else F::template run<-1>(v, lds, ph, twp<T>(g, 0));
#pragma unroll
    for (int i = 0; i < F::template nout<-1>(); ++i) {
        int p, e;
        if (F::template out_pos<-1>(i, p, e)) split[F::lidx(p, e)] = v[i];
    }
    F::sync();
    split_rows<T, L, F>(split, reinterpret_cast<cx<T> *>(a.spec) + (long long)f * g.NC, pair0, Pact, rows);
}

// X3: half spectra of E_k (species blockIdx.y) -> inverse x -> Euler-Lagrange update
// G = rho_b exp(base + E) (eq. rhoEquation) and the weighted residual sums; raw mode
// writes E (+ addend) only.
template <typename T, int L>
__global__ __launch_bounds__(XTile<L>::NTB) void k_x3c(Geo g_in, X3Args a) {
    using XT = XTile<L>;
    constexpr int PB = XT::PB, NTB = XT::NTB, KX = XT::KX;
    using F = ct::Fft<T, typename ct::XPlan<L>::type, PB, NTB, true, 2, XT::PAD>;
    const int prob = (int)blockIdx.z;
    if (prob > 0) {
        const long long o = (long long)prob * g_in.pstride;
        g_in = shift(g_in, o);
        a = shift(a, o);
    }
    const Geo &g = g_in;
    if (gated_off(a.gate)) return;
    resolve_roles(a);
    // wave-private tiles: twiddles fetched up front, with the data
    typename F::Twiddles trw;
    if constexpr (F::WP) F::load_twiddles(trw, twp<T>(g_in, 0));
    __shared__ cx<T> lds[F::LDS_ELEMS];
    const Consts &c = *g.cs;
    const int sp = blockIdx.y;
    const long long N = g.N;
    const long long rows = (long long)g.ny * g.nz;
    const long long npairs = (rows + 1) / 2;
    const long long pair0 = (long long)blockIdx.x * PB;
    const int Pact = (int)min((long long)PB, npairs - pair0);
    const cx<T> *in = reinterpret_cast<const cx<T> *>(a.specA) + (long long)sp * g.NC;
    cx<T> v[F::V];
    load_row_pairs<T, L, F>(in, pair0, Pact, rows, v);
    int ph = 0;
    if constexpr (F::WP) F::template run<1>(v, lds, ph, trw);
    else F::template run<1>(v, lds, ph, twp<T>(g, 0));
    double acc = 0.0;
    int flag = 0;
    const double rb = c.rho_b[sp], irb = c.inv_rho_b[sp], zs = c.z[sp];
#pragma unroll
    for (int i = 0; i < F::template nout<1>(); ++i) {
        int p, e;
        if (!(F::template out_pos<1>(i, p, e) && p < Pact)) continue;
        const long long r0 = 2 * (pair0 + p);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long r = r0 + h;
            if (r >= rows) break;
            const double E = h == 0 ? (double)v[i].x : (double)v[i].y;
            const long long node = r * L + e;
            const long long idx = (long long)sp * N + node;
            if (a.raw) {
                double o = E;
                if (a.addend) o += ct::gld(a.addend + node);
                ct::gst(a.raw_out + idx, o);
                continue;
            }
            const double b = ct::cld(a.base + idx);
            const bool fluid = b > -INFINITY;
            const double G = fluid ? rb * exp(b + E) : 0.0;
            if (a.g_out) ct::gst(a.g_out + idx, G);
            if (a.e_out) ct::gst(a.e_out + idx, a.e_phi ? E - zs * ct::gld(a.e_phi + node) : E);
            if (a.lp_out) ct::gst(a.lp_out + idx, fluid ? b + E : -INFINITY);
            if (fluid) {
                const double dlt = (ct::cld(a.rho_t + idx) - G) * irb;
                acc += dlt * dlt;
                if (!isfinite(G)) flag |= 1;
            }
        }
    }
    if (a.raw) return;
    const long long slot = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    block_reduce_nt<false, NTB>(acc, flag, a.red.fpart + slot, a.red.fflag + slot);
}

}  // namespace dft
