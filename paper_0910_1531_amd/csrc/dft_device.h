// Device building blocks for gfx950: complex arithmetic, the LDS-staged mixed-radix
// Stockham FFT used by every pass kernel, the analytic spectra of Appendix B and of the
// bulk-fluid section, and the pointwise derivatives of eq. (Phi).
#pragma once

#include <hip/hip_runtime.h>

#include "dft_host.h"

namespace dft {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk<T>(a.x, -a.y); }
// multiply by s*i (s = +1 or -1)
template <typename T, int SGN>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return SGN > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x); }

// ------------------------------------------------------------------ FFT plan on device
struct DevPlan {
    int L;
    int nr;
    int r[kMaxRadices];
};

// ------------------------------------------------------------------ radix butterflies
// X_m = sum_q v_q exp(DIR 2 pi i q m / R), in place.
template <typename T, int DIR>
__device__ __forceinline__ void bfly2(cx<T> *v) {
    cx<T> a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly4(cx<T> *v) {
    cx<T> t0 = add(v[0], v[2]), t1 = sub(v[0], v[2]);
    cx<T> t2 = add(v[1], v[3]), t3 = mul_i<T, DIR>(sub(v[1], v[3]));
    v[0] = add(t0, t2);
    v[2] = sub(t0, t2);
    v[1] = add(t1, t3);
    v[3] = sub(t1, t3);
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly3(cx<T> *v) {
    const T c = T(-0.5);
    const T s = T(DIR) * T(0.86602540378443864676372317075293618);
    cx<T> a = v[0];
    cx<T> sm = add(v[1], v[2]);
    cx<T> df = sub(v[1], v[2]);
    v[0] = add(a, sm);
    cx<T> m = mk<T>(a.x + c * sm.x, a.y + c * sm.y);
    cx<T> r = mk<T>(-s * df.y, s * df.x);   // i s (b - c)
    v[1] = add(m, r);
    v[2] = sub(m, r);
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly8(cx<T> *v) {
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    bfly4<T, DIR>(e);
    bfly4<T, DIR>(o);
    const T r2 = T(0.70710678118654752440084436210484903);
    // o[m] *= exp(DIR 2 pi i m / 8)
    o[1] = mk<T>(r2 * (o[1].x - T(DIR) * o[1].y), r2 * (o[1].y + T(DIR) * o[1].x));
    o[2] = mul_i<T, DIR>(o[2]);
    o[3] = mk<T>(r2 * (-o[3].x - T(DIR) * o[3].y), r2 * (-o[3].y + T(DIR) * o[3].x));
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        v[m] = add(e[m], o[m]);
        v[m + 4] = sub(e[m], o[m]);
    }
}

template <typename T, int DIR, int R>
__device__ __forceinline__ void bfly(cx<T> *v) {
    if constexpr (R == 2) bfly2<T, DIR>(v);
    else if constexpr (R == 3) bfly3<T, DIR>(v);
    else if constexpr (R == 4) bfly4<T, DIR>(v);
    else bfly8<T, DIR>(v);
}

// ------------------------------------------------------------------ Stockham stage in LDS
// The tile holds P pencils of length L; element e of pencil p is tile[p*ps + e*es].
// One stage of radix R: butterfly b of a pencil reads elements b + q*L/R, applies the
// twiddles exp(DIR 2 pi i q k / (Ns R)) with k = b mod Ns, and writes the outputs to
// (b / Ns) * Ns * R + k + q * Ns.  Every thread reads all of its inputs before the
// barrier and writes after it, so the stage runs in place.
// `bfast` selects the butterfly index as the fastest-varying work index (x tiles,
// es == 1); otherwise the pencil index varies fastest (y/z tiles, ps == 1).
template <typename T, int DIR, int R, int NT, int MAXE>
__device__ __forceinline__ void stockham_stage(cx<T> *tile, int L, int P, int es, int ps, bool bfast, int Ns,
                                               const cx<T> *__restrict__ tw) {
    constexpr int IT = (MAXE + R - 1) / R;
    const int nb = L / R;
    const int total = nb * P;
    const int tstride = L / (Ns * R);
    cx<T> v[IT][R];
    int obase[IT];
    int kk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int j = threadIdx.x + it * NT;
        if (j < total) {
            int p, b;
            if (bfast) { b = j % nb; p = j / nb; }
            else { p = j % P; b = j / P; }
            const int ib = p * ps + b * es;
#pragma unroll
            for (int q = 0; q < R; ++q) v[it][q] = tile[ib + q * nb * es];
            const int k = b % Ns;
            kk[it] = k;
            obase[it] = p * ps + ((b - k) * R + k) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int j = threadIdx.x + it * NT;
        if (j < total) {
            const int k = kk[it];
            if (Ns > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    cx<T> w = tw[q * k * tstride];
                    if (DIR > 0) w.y = -w.y;
                    v[it][q] = mul(v[it][q], w);
                }
            }
            bfly<T, DIR, R>(v[it]);
#pragma unroll
            for (int q = 0; q < R; ++q) tile[obase[it] + q * Ns * es] = v[it][q];
        }
    }
    __syncthreads();
}

// Full FFT of every pencil in the tile (unnormalized; DIR = -1 forward, +1 inverse).
// Requires L * P <= NT * MAXE (checked by the launchers).
template <typename T, int DIR, int NT, int MAXE>
__device__ __forceinline__ void fft_tile(cx<T> *tile, const DevPlan &pl, int P, int es, int ps, bool bfast,
                                         const cx<T> *__restrict__ tw) {
    int Ns = 1;
    for (int s = 0; s < pl.nr; ++s) {
        const int R = pl.r[s];
        if (R == 8) stockham_stage<T, DIR, 8, NT, MAXE>(tile, pl.L, P, es, ps, bfast, Ns, tw);
        else if (R == 4) stockham_stage<T, DIR, 4, NT, MAXE>(tile, pl.L, P, es, ps, bfast, Ns, tw);
        else if (R == 2) stockham_stage<T, DIR, 2, NT, MAXE>(tile, pl.L, P, es, ps, bfast, Ns, tw);
        else stockham_stage<T, DIR, 3, NT, MAXE>(tile, pl.L, P, es, ps, bfast, Ns, tw);
        Ns *= R;
    }
}

template <typename T, int NT, int MAXE>
__device__ __forceinline__ void fft_tile_dir(int dir, cx<T> *tile, const DevPlan &pl, int P, int es, int ps,
                                             bool bfast, const cx<T> *__restrict__ tw) {
    if (dir < 0) fft_tile<T, -1, NT, MAXE>(tile, pl, P, es, ps, bfast, tw);
    else fft_tile<T, 1, NT, MAXE>(tile, pl, P, es, ps, bfast, tw);
}

// ------------------------------------------------------------------ spectra (FP64)
// Series of (4 pi / k) I_m(R, k) / (4 pi R^{m+3}) = sum_n (-1)^n y^{2n} / ((2n+1)! (2n+m+3)),
// y = kR, used below y = 1 where the closed forms lose digits.
constexpr int kSeriesTerms = 11;

template <int M>
struct BallSeries {
    double c[kSeriesTerms];
    constexpr BallSeries() : c() {
        double fact = 1.0;   // (2n+1)!
        for (int n = 0; n < kSeriesTerms; ++n) {
            if (n > 0) fact *= (double)(2 * n) * (double)(2 * n + 1);
            c[n] = ((n % 2) ? -1.0 : 1.0) / (fact * (double)(2 * n + M + 3));
        }
    }
};

struct SincSeries {   // sin(y)/y = sum (-1)^n y^{2n} / (2n+1)!
    double c[kSeriesTerms];
    constexpr SincSeries() : c() {
        double fact = 1.0;
        for (int n = 0; n < kSeriesTerms; ++n) {
            if (n > 0) fact *= (double)(2 * n) * (double)(2 * n + 1);
            c[n] = ((n % 2) ? -1.0 : 1.0) / fact;
        }
    }
};

// Series in y^2 for y < 1.  FP32 (differences from an FP64 reference) stops after six
// terms: the first omitted one is at most 2e-10 of the sum.
template <typename R, typename S>
__device__ __forceinline__ R horner_y2(const S &s, R y2) {
    constexpr int nt = sizeof(R) == 4 ? 6 : kSeriesTerms;
    R acc = R(s.c[nt - 1]);
#pragma unroll
    for (int n = nt - 2; n >= 0; --n) acc = fma(acc, y2, R(s.c[n]));
    return acc;
}

constexpr double kFourPi = 12.566370614359172953850573533118011536788677597500;

__device__ __forceinline__ void sincos_r(double y, double *s, double *c) { sincos(y, s, c); }
__device__ __forceinline__ void sincos_r(float y, float *s, float *c) { sincosf(y, s, c); }
// Sine and cosine of the spectral weights' arguments k R (at most a few tens of radians): FP64
// as sincos; FP32 (weights of difference spectra) by the hardware's sine and cosine of the
// argument in revolutions reduced to [0, 1), which adds an absolute error of a few 1e-7 to the
// argument's own rounding.
__device__ __forceinline__ void sincos_w(double y, double *s, double *c) { sincos(y, s, c); }
__device__ __forceinline__ void sincos_w(float y, float *s, float *c) {
    const float r = __builtin_amdgcn_fractf(y * 0.159154943091895336f);   // y / (2 pi)
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}

// Reciprocal and square root in the arithmetic type: IEEE operations in FP64; in FP32 the
// hardware's single-instruction approximations (about 1 ulp), enough for the spectral factors
// that multiply FP32 difference spectra.
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }

// Weight transforms of a sphere of radius R at |k| (Appendix B):
//   w2 = 4 pi R sin(kR) / k,   w3 = 4 pi (sin kR - kR cos kR) / k^3,
// given s = sin(kR) and c = cos(kR) (used only for kR >= 1; the series covers kR < 1).
// R is the arithmetic type (double for FP64 evaluations, float for FP32 differences).
template <typename R>
__device__ __forceinline__ void weight_w2_w3_sc(R k, R Rad, R s, R c, R &w2, R &w3) {
    const R y = k * Rad;
    const R R2 = Rad * Rad;
    if (y < R(1)) {
        constexpr SincSeries s0{};
        constexpr BallSeries<0> s3{};
        const R y2 = y * y;
        w2 = R(kFourPi) * R2 * horner_y2<R>(s0, y2);
        w3 = R(kFourPi) * R2 * Rad * horner_y2<R>(s3, y2);
    } else {
        const R iy = rcp_r(y);
        w2 = R(kFourPi) * R2 * s * iy;
        w3 = R(kFourPi) * R2 * Rad * (s - y * c) * iy * iy * iy;
    }
}

template <typename R>
__device__ __forceinline__ void weight_w2_w3(R k, R Rad, R &w2, R &w3) {
    R s = R(0), c = R(1);
    if (k * Rad >= R(1)) sincos_w(k * Rad, &s, &c);
    weight_w2_w3_sc<R>(k, Rad, s, c, w2, w3);
}

// Transform of the unit-mean ball indicator of radius R at |k| (the screening kernel of the RFD
// section, eq. screening-kernel-hat): 3 (sin kR - kR cos kR) / (kR)^3 = w3 / (4 pi R^3 / 3).
template <typename R>
__device__ __forceinline__ R ball_mean(R k, R Rad) {
    R w2, w3;
    weight_w2_w3<R>(k, Rad, w2, w3);
    return w3 * R(3.0 / kFourPi) / (Rad * Rad * Rad);
}

// Bulk-fluid kernel transform for one pair: c1 F1 + c0 F0 + cm1 Fm1 with
// F_m = integral over |r| <= Rc of r^m exp(-i k.r) = (4 pi / k) I_m(Rc, k),
// given s = sin(k Rc), c = cos(k Rc) (used for k Rc >= 1).
template <typename R>
__device__ __forceinline__ R screening_hat_sc(R k, R Rc, R s, R c, R c1, R c0, R cm1) {
    const R y = k * Rc;
    const R R2 = Rc * Rc;
    R Fm1, F0, F1;
    if (y < R(1)) {
        constexpr BallSeries<-1> sm{};
        constexpr BallSeries<0> s0{};
        constexpr BallSeries<1> s1{};
        const R y2 = y * y;
        Fm1 = R(kFourPi) * R2 * horner_y2<R>(sm, y2);
        F0 = R(kFourPi) * R2 * Rc * horner_y2<R>(s0, y2);
        F1 = R(kFourPi) * R2 * R2 * horner_y2<R>(s1, y2);
    } else {
        const R omc = (c > R(0)) ? s * s * rcp_r(R(1) + c) : R(1) - c;   // 1 - cos y without cancellation
        const R iy = rcp_r(y), iy2 = iy * iy;
        Fm1 = R(kFourPi) * R2 * omc * iy2;
        F0 = R(kFourPi) * R2 * Rc * (s - y * c) * iy2 * iy;
        F1 = R(kFourPi) * R2 * R2 * (-c * iy2 + R(2) * s * iy2 * iy - R(2) * omc * iy2 * iy2);
    }
    return c1 * F1 + c0 * F0 + cm1 * Fm1;
}

// The same factor from the regrouped pair constants p1..p4 (a = -p4 / 2, b = p2 + p4, g = p3):
//   k Rc >= 1:  (p1 c + p2 s / y + (1 - c)(p3 + p4 / y^2)) / y^2,
//   k Rc < 1:   a S1(y) + b S0(y) + g Sm1(y) with the series of F1, F0, Fm1 over their prefactors.
template <typename R>
__device__ __forceinline__ R screening_hat_p(R k, R Rc, R s, R c, R p1, R p2, R p3, R p4) {
    const R y = k * Rc;
    if (y < R(1)) {
        constexpr BallSeries<-1> sm{};
        constexpr BallSeries<0> s0{};
        constexpr BallSeries<1> s1{};
        const R y2 = y * y;
        return R(-0.5) * p4 * horner_y2<R>(s1, y2) + (p2 + p4) * horner_y2<R>(s0, y2) + p3 * horner_y2<R>(sm, y2);
    }
    const R omc = (c > R(0)) ? s * s * rcp_r(R(1) + c) : R(1) - c;   // 1 - cos y without cancellation
    const R iy = rcp_r(y), iy2 = iy * iy;
    return iy2 * (p1 * c + p2 * s * iy + omc * (p3 + p4 * iy2));
}

template <typename R>
__device__ __forceinline__ R screening_hat(R k, R Rc, R c1, R c0, R cm1) {
    R s = R(0), c = R(1);
    if (k * Rc >= R(1)) sincos_r(k * Rc, &s, &c);
    return screening_hat_sc<R>(k, Rc, s, c, c1, c0, cm1);
}

// 2 (1 - cos t) = 4 sin^2(t / 2) from (cos t, +-sin t) without cancellation.
template <typename R>
__device__ __forceinline__ R two_omc(R c, R s) {
    return (c > R(0)) ? R(2) * s * s * rcp_r(R(1) + c) : R(2) * (R(1) - c);
}

// Eigenvalue of minus the 7-point Laplacian for wavenumber components kd.
template <typename R>
__device__ __forceinline__ R poisson_denominator(const R kd[3], const double h[3]) {
    R D = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R hd = R(h[d]);
        R s, c;
        sincos_r(R(0.5) * kd[d] * hd, &s, &c);
        D += R(4) * s * s / (hd * hd);
    }
    return D;
}

// Signed mode index of position j on an axis with n nodes (eq. Kvalues).
__device__ __forceinline__ int signed_mode(int j, int n) { return (2 * j <= n) ? j : j - n; }

// Wavenumber data of one element of a z tile.
struct KInfo {
    double k[3];
    double kmag;
    bool nyq[3];
    bool zero;
};

__device__ __forceinline__ KInfo kinfo(const Consts &c, int jx, int y, int e) {
    KInfo q;
    const int my = signed_mode(y, c.ny), mz = signed_mode(e, c.nz);
    q.k[0] = jx * c.dk[0];
    q.k[1] = my * c.dk[1];
    q.k[2] = mz * c.dk[2];
    q.kmag = sqrt(q.k[0] * q.k[0] + q.k[1] * q.k[1] + q.k[2] * q.k[2]);
    q.nyq[0] = (c.nx % 2 == 0) && (2 * jx == c.nx);
    q.nyq[1] = (c.ny % 2 == 0) && (2 * y == c.ny);
    q.nyq[2] = (c.nz % 2 == 0) && (2 * e == c.nz);
    q.zero = (jx == 0) && (y == 0) && (e == 0);
    return q;
}

// Component d of k, zero on the Nyquist plane of axis d (register selects, no indexing).
__device__ __forceinline__ double k_comp(const KInfo &q, int d) {
    const double k = d == 0 ? q.k[0] : (d == 1 ? q.k[1] : q.k[2]);
    const bool ny = d == 0 ? q.nyq[0] : (d == 1 ? q.nyq[1] : q.nyq[2]);
    return ny ? 0.0 : k;
}

// Ball moments F_m = integral over |r| <= Rc of r^m exp(-i k.r), m = 1, 0, -1, and j0(k Rc).
__device__ __forceinline__ void ball_moments(double k, double Rc, double &F1, double &F0, double &Fm1, double &j0) {
    const double y = k * Rc;
    const double R2 = Rc * Rc;
    if (y < 1.0) {
        constexpr BallSeries<-1> sm{};
        constexpr BallSeries<0> s0{};
        constexpr BallSeries<1> s1{};
        constexpr SincSeries sj{};
        const double y2 = y * y;
        Fm1 = kFourPi * R2 * horner_y2<double>(sm, y2);
        F0 = kFourPi * R2 * Rc * horner_y2<double>(s0, y2);
        F1 = kFourPi * R2 * R2 * horner_y2<double>(s1, y2);
        j0 = horner_y2<double>(sj, y2);
    } else {
        double s, c;
        sincos(y, &s, &c);
        const double omc = (c > 0.0) ? s * s / (1.0 + c) : 1.0 - c;
        const double iy = 1.0 / y, iy2 = iy * iy;
        Fm1 = kFourPi * R2 * omc * iy2;
        F0 = kFourPi * R2 * Rc * (s - y * c) * iy2 * iy;
        F1 = kFourPi * R2 * R2 * (-c * iy2 + 2.0 * s * iy2 * iy - 2.0 * omc * iy2 * iy2);
        j0 = s * iy;
    }
}

// ------------------------------------------------------------------ eq. (Phi)
// dPhi/dn_alpha of the anti-symmetrized Rosenfeld free-energy density, with the
// bound |nV2| <= n2 enforced as xi^2 <- min(xi^2, 1).  D may be double or a dual number.
template <typename D>
struct FmtOps;

template <>
struct FmtOps<double> {
    static __device__ __forceinline__ double val(double a) { return a; }
    static __device__ __forceinline__ double cst(double a) { return a; }
    static __device__ __forceinline__ double lg(double a) { return log(a); }
    // a scalar function g of x given g(x) and g'(x): the value (duals also carry g'(x) dx)
    static __device__ __forceinline__ double fn(double, double g, double) { return g; }
};

// Forward-mode dual number: value and derivative along one direction.  fmt_dphi on duals
// returns dPhi/dn at the value and the Hessian-vector product Phi''(n) dn in the tangent.
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}

template <>
struct FmtOps<Dual> {
    static __device__ __forceinline__ double val(Dual a) { return a.v; }
    static __device__ __forceinline__ Dual cst(double a) { return {a, 0.0}; }
    static __device__ __forceinline__ Dual lg(Dual a) { return {log(a.v), a.d / a.v}; }
    static __device__ __forceinline__ Dual fn(Dual x, double g, double gp) { return {g, gp * x.d}; }
};

template <typename D>
__device__ __forceinline__ void fmt_dphi(const D n[DFT_NALPHA], D out[DFT_NALPHA], bool &clamped) {
    using O = FmtOps<D>;
    const double inv8pi = 1.0 / (8.0 * 3.14159265358979323846);
    const double inv12pi = 1.0 / (12.0 * 3.14159265358979323846);
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
    const D one = O::cst(1.0);
    const D Dm = one - n[3];
    const D iD = one / Dm;
    const D dot12 = n[4] * n[7] + n[5] * n[8] + n[6] * n[9];
    const D dot22 = n[7] * n[7] + n[8] * n[8] + n[9] * n[9];
    const D n2sq = n[2] * n[2];
    const D den = (O::val(n2sq) > 1e-300) ? n2sq : O::cst(1e-300);
    D x2 = dot22 / den;
    clamped = !(O::val(x2) < 1.0);
    if (clamped) x2 = one;
    const D q = one - x2;
    const D q2 = q * q;
    const D iD2 = iD * iD;
    out[0] = O::cst(0.0) - O::lg(Dm);
    out[1] = n[2] * iD;
    out[2] = n[1] * iD + n2sq * q2 * (one + x2) * iD2 * inv8pi;
    out[3] = n[0] * iD + (n[1] * n[2] - dot12) * iD2 + n2sq * n[2] * q2 * q * iD2 * iD * inv12pi;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out[4 + d] = O::cst(0.0) - n[7 + d] * iD;
        out[7 + d] = O::cst(0.0) - n[4 + d] * iD - n[2] * q2 * n[7 + d] * iD2 * inv4pi;
    }
}


// ------------------------------------------------------------------ alternative Phi
// Functionals that keep the first two terms of eq. (Phi) and replace the third by
// (n2^3 - 3 n2 nV2.nV2) f(n3) / (36 pi): Rosenfeld's original vector form, f = 3 / (2 (1 - n3)^2),
// and White Bear, f = (n3 + (1 - n3)^2 ln(1 - n3)) / (n3^2 (1 - n3)^2), whose bulk is the BMCSL
// equation of state.  The bound |nV2| <= n2 is applied as nV2.nV2 <- min(nV2.nV2, n2^2).

// White Bear f and its first two derivatives.  The closed forms cancel as n3 -> 0 (f -> 3/2);
// below |n3| = 0.1 the Taylor series f = sum_k (k+1)(k+3)/(k+2) n3^k is summed instead (24 terms:
// the remainder of f'' is below 1e-17 there).  Above, with L = ln(1 - x) and y = 1 - x:
//   f'  = -2 L / x^3 - (x^2 - 5 x + 2) / (x^2 y^3)
//   f'' =  6 L / x^4 + (-5 x^3 + 26 x^2 - 21 x + 6) / (x^3 y^4)
__device__ __forceinline__ void wb_factor(double x, double &f0, double &f1, double &f2) {
    if (fabs(x) < 0.1) {
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int k = 23; k >= 0; --k) {
            const double ck = (double)((k + 1) * (k + 3)) / (double)(k + 2);
            c = c * x + 2.0 * b;   // running second derivative of the partial sum
            b = b * x + a;
            a = a * x + ck;
        }
        f0 = a;
        f1 = b;
        f2 = c;
        return;
    }
    const double y = 1.0 - x, L = log1p(-x);
    const double ix = 1.0 / x, iy = 1.0 / y;
    const double ix2 = ix * ix, iy2 = iy * iy;
    f0 = (x + y * y * L) * ix2 * iy2;
    f1 = -2.0 * L * ix2 * ix - (x * x - 5.0 * x + 2.0) * ix2 * iy2 * iy;
    f2 = 6.0 * L * ix2 * ix2 + (((-5.0 * x + 26.0) * x - 21.0) * x + 6.0) * ix2 * ix * iy2 * iy2;
}

// dPhi/dn of the alternative forms; hs = DFT_HS_ROSENFELD or DFT_HS_WHITE_BEAR.
template <typename D>
__device__ __forceinline__ void fmt_dphi_alt(int hs, const D n[DFT_NALPHA], D out[DFT_NALPHA], bool &clamped) {
    using O = FmtOps<D>;
    const double inv36pi = 1.0 / (36.0 * 3.14159265358979323846);
    const D one = O::cst(1.0);
    const D Dm = one - n[3];
    const D iD = one / Dm;
    const D dot12 = n[4] * n[7] + n[5] * n[8] + n[6] * n[9];
    const D dot22 = n[7] * n[7] + n[8] * n[8] + n[9] * n[9];
    const D n2sq = n[2] * n[2];
    const double den = O::val(n2sq) > 1e-300 ? O::val(n2sq) : 1e-300;
    clamped = !(O::val(dot22) / den < 1.0);
    const D g = clamped ? n2sq : dot22;   // nV2.nV2 after the bound
    D f, fp;
    if (hs == DFT_HS_WHITE_BEAR) {
        double f0, f1, f2;
        wb_factor(O::val(n[3]), f0, f1, f2);
        f = O::fn(n[3], f0, f1);
        fp = O::fn(n[3], f1, f2);
    } else {
        const D iD2 = iD * iD;
        f = iD2 * 1.5;
        fp = iD2 * iD * 3.0;
    }
    // d/dn2 of (n2^3 - 3 n2 g): 3 n2^2 - 3 g, or -6 n2^2 where g = n2^2 (bound active)
    const D dn2 = clamped ? n2sq * (-6.0) : (n2sq - g) * 3.0;
    const D third = n[2] * (n2sq - g * 3.0);
    out[0] = O::cst(0.0) - O::lg(Dm);
    out[1] = n[2] * iD;
    out[2] = n[1] * iD + dn2 * f * inv36pi;
    out[3] = n[0] * iD + (n[1] * n[2] - dot12) * iD * iD + third * fp * inv36pi;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out[4 + d] = O::cst(0.0) - n[7 + d] * iD;
        out[7 + d] = O::cst(0.0) - n[4 + d] * iD;
        if (!clamped) out[7 + d] = out[7 + d] - n[2] * n[7 + d] * f * (6.0 * inv36pi);
    }
}

// dPhi/dn of the functional hs (dft_hs_functional), chosen at run time.
template <typename D>
__device__ __forceinline__ void fmt_dphi_sel(int hs, const D n[DFT_NALPHA], D out[DFT_NALPHA], bool &clamped) {
    if (hs == DFT_HS_RSLT) fmt_dphi<D>(n, out, clamped);
    else fmt_dphi_alt<D>(hs, n, out, clamped);
}

// Compile-time choice for kernels instantiated per family: ALT = false compiles eq. (Phi) only,
// ALT = true the alternative forms only (hs picks between them).
template <bool ALT, typename D>
__device__ __forceinline__ void fmt_dphi_as(int hs, const D n[DFT_NALPHA], D out[DFT_NALPHA], bool &clamped) {
    if constexpr (ALT) fmt_dphi_alt<D>(hs, n, out, clamped);
    else fmt_dphi<D>(n, out, clamped);
}

}  // namespace dft
