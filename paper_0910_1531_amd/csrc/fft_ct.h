// Compile-time-length Stockham FFT over LDS tiles of pencils, for gfx950.
//
// A tile holds P pencils of length L.  Each thread owns whole butterflies: the stage of
// radix R has L P / R butterflies spread over the NT threads of the block, and a thread
// keeps the R values of each of its butterflies in registers.  Between stages the values
// go through one of two LDS buffers used in turn, so each exchange needs one barrier (a
// wave-level fence only, where every wave owns whole pencils: see wave_private).
// The first stage takes its inputs from registers that the caller filled (straight from
// HBM) and the last stage leaves its outputs in registers (stored straight to HBM), so a
// transform costs (stages - 1) LDS round trips.  The inverse transform runs the radices
// in reverse order: the positions a thread holds after the last forward stage are then the
// positions the first inverse stage needs, and a kernel can apply a spectral product in
// registers between a forward and an inverse transform.
//
// With L, P, NT and the radices fixed at compile time every index is a constant or a
// shift, and the stage loop unrolls completely (no run-time plan, no scratch memory).
// Twiddles are read from the per-axis table at each stage, or, for blocks that run several
// transforms in one direction, loaded once into registers (TwReg, or Twiddles for
// wave-private tiles, which serve both directions).
#pragma once

#include "dft_device.h"

namespace dft {
namespace ct {

// ---------------------------------------------------------------- global-memory access
// Loads and stores through the global address space (not flat), so LDS waits never wait
// for HBM traffic.
template <typename T> struct V2 { typedef T type __attribute__((ext_vector_type(2))); };

template <typename T>
__device__ __forceinline__ cx<T> gld(const cx<T> *p) {
    typedef __attribute__((address_space(1))) const typename V2<T>::type *GP;
    const typename V2<T>::type r = *(GP)p;
    return mk<T>(r.x, r.y);
}
template <typename T>
__device__ __forceinline__ void gst(cx<T> *p, cx<T> v) {
    typedef __attribute__((address_space(1))) typename V2<T>::type *GP;
    typename V2<T>::type r;
    r.x = v.x;
    r.y = v.y;
    *(GP)p = r;
}
template <typename T>
__device__ __forceinline__ T gld(const T *p) {
    return *(__attribute__((address_space(1))) const T *)p;
}
template <typename T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}
// Loads of data that no thread writes while the kernel runs (twiddles, spectral tables, the
// reference fields): through the constant address space, so the compiler knows no store of the
// kernel changes them and may issue them ahead of earlier stores.
template <typename T>
__device__ __forceinline__ cx<T> cld(const cx<T> *p) {
    typedef __attribute__((address_space(4))) const typename V2<T>::type *CP;
    const typename V2<T>::type r = *(CP)p;
    return mk<T>(r.x, r.y);
}
template <typename T>
__device__ __forceinline__ T cld(const T *p) {
    return *(__attribute__((address_space(4))) const T *)p;
}

// ---------------------------------------------------------------- radix schedules
// Radices in the order the forward transform runs them.
template <int... Rs>
struct Sched {
    static constexpr int n = sizeof...(Rs);
    static constexpr int L = (1 * ... * Rs);
    static constexpr int r(int s) {
        constexpr int a[] = {Rs...};
        return a[s];
    }
};

// ---------------------------------------------------------------- the engine
// XOR swizzle of the element index within an x pencil in LDS.  The radix-4 Stockham
// writes of the first stages go to elements 4 l + q and 16 (b / 4) + b % 4 + 4 q for lanes
// l, b; mixing bits above the bank-group width (128 bytes = 16 complex floats or 8 complex
// doubles) into the low bits gives the lanes of one LDS access cycle distinct bank groups,
// while contiguous reads stay contiguous.  The map is a bijection on each aligned block.
template <typename T>
__host__ __device__ constexpr int xswz(int e) {
    if constexpr (sizeof(T) == 4) {
        const int h = (e >> 4) & 3;
        return e ^ (h | (h << 2));
    } else {
        return e ^ (((e >> 3) & 3) | (((e >> 4) & 1) << 2));
    }
}
template <typename T>
constexpr bool xswz_fits(int L) {
    for (int e = 0; e < L; ++e)
        if (xswz<T>(e) >= L) return false;
    return true;
}

// Row swizzle of y and z tiles (pencil index fastest: LDS row e holds element e of the P
// pencils).  LDS serves 128 bytes per cycle, sixteen 8-byte or eight 16-byte lanes.  Rows of
// 64 or 32 bytes put two or four rows in one cycle's lanes, and the Stockham writes of the
// early stages send those lanes to rows a multiple of 4 or 8 apart, which sit on the same
// banks.  XOR-ing higher bits of the row index into its low bit (64-byte rows) or two low
// bits (32-byte rows) spreads them over distinct banks; the bits are chosen per length by an
// exhaustive search over this access model (power-of-two lengths: no conflicts left in either
// direction).  Rows of 128 bytes or more are not swizzled.  A bijection on each aligned
// block of 2 or 4 rows, so rows stay inside [0, L).
template <int L, int ROWB>
__host__ __device__ constexpr int yzswz(int e) {
    constexpr bool pow2 = (L & (L - 1)) == 0;
    const int b2 = (e >> 2) & 1, b3 = (e >> 3) & 1, b4 = (e >> 4) & 1, b5 = (e >> 5) & 1;
    if constexpr (ROWB == 64) {
        if constexpr (pow2 || L == 48) return e ^ (b2 ^ b3);
        else if constexpr (L == 24 || L == 192) return e ^ (b3 ^ b4);
        else return e ^ b3;
    } else if constexpr (ROWB == 32) {
        int x = 0, y = 0;
        if constexpr (pow2) { x = b2 ^ b3; y = b3 ^ b4; }
        else if constexpr (L == 24) { x = b3; y = b3 ^ b4; }
        else if constexpr (L == 48) { x = b2; y = b3 ^ b4; }
        else if constexpr (L == 192) { x = b3 ^ b4; y = b3 ^ b5; }
        else { x = b3 ^ b5; y = b3 ^ b4; }
        return e ^ (x | (y << 1));
    } else {
        return e;
    }
}
template <int L, int ROWB>
constexpr bool yzswz_ok() {
    bool seen[L] = {};
    for (int e = 0; e < L; ++e) {
        const int f = yzswz<L, ROWB>(e);
        if (f < 0 || f >= L || seen[f]) return false;
        seen[f] = true;
    }
    return true;
}

// BF = false: the pencil index varies fastest over threads and in LDS (y and z tiles,
// whose pencils are adjacent columns in HBM).  BF = true: the element index varies fastest
// (x tiles, whose pencils are rows); elements are swizzled (xswz) against bank conflicts.
// NB = 2 alternates two LDS buffers (one barrier per exchange); NB = 1 uses one buffer and
// a second barrier before each write.
template <typename T, class SC, int P, int NT, bool BF, int NB = 2, int PAD = 0>
struct Fft {
    static constexpr int L = SC::L;
    static constexpr int NSTG = SC::n;
    static constexpr int LS = BF ? L + PAD : L;
    static constexpr int TILE = BF ? P * (L + PAD) : L * P;   // LDS elements per buffer
    static constexpr int LDS_ELEMS = NB * TILE;

    template <int DIR>
    static constexpr int rad(int s) { return DIR < 0 ? SC::r(s) : SC::r(NSTG - 1 - s); }
    // product of the radices before stage s
    template <int DIR>
    static constexpr int span(int s) {
        int m = 1;
        for (int i = 0; i < s; ++i) m *= rad<DIR>(i);
        return m;
    }
    static constexpr int items(int R) { return L * P / R; }
    static constexpr int iters(int R) { return (items(R) + NT - 1) / NT; }
    static constexpr bool exact(int R) { return items(R) % NT == 0; }
    static constexpr int regs(int R) { return iters(R) * R; }
    static constexpr int vmax() {
        int m = 0;
        for (int s = 0; s < NSTG; ++s) m = regs(SC::r(s)) > m ? regs(SC::r(s)) : m;
        return m;
    }
    static constexpr int V = vmax();   // registers (complex values) per thread
    // Wave-private tiles: every stage radix 4 with exactly one butterfly per thread, and whole
    // pencils per wave (L / 4 divides 64).  Each wave then reads and writes only its own pencils'
    // LDS regions, and the LDS instructions of one wave execute in order, so a wave-level fence
    // (compiler and memory ordering within the wavefront) replaces the block barrier.
    static constexpr bool wave_private() {
        if (!BF) return false;
        for (int s = 0; s < NSTG; ++s)
            if (SC::r(s) != 4) return false;
        return items(4) == NT && NT % 64 == 0 && 64 % (L / 4) == 0;
    }
    static constexpr bool WP = wave_private();
    __device__ static __forceinline__ void sync() {
        if constexpr (WP) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    }

    template <int DIR> static constexpr int nin() { return regs(rad<DIR>(0)); }
    template <int DIR> static constexpr int nout() { return regs(rad<DIR>(NSTG - 1)); }

    // butterfly j of a radix-R stage -> pencil p and butterfly index b within the pencil
    template <int R>
    __device__ static __forceinline__ void decode(int j, int &p, int &b) {
        constexpr int nb = L / R;
        if constexpr (BF) {
            p = j / nb;
            b = j - p * nb;
        } else {
            b = j / P;
            p = j - b * P;
        }
    }
    static_assert(!BF || xswz_fits<T>(L), "swizzle leaves the pencil");
    static constexpr int ROWB = P * (int)sizeof(cx<T>);
    static_assert(BF || yzswz_ok<L, ROWB>(), "row swizzle is not a permutation");
    __device__ static __forceinline__ int lidx(int p, int e) {
        if constexpr (BF) return p * LS + xswz<T>(e);
        else return yzswz<L, ROWB>(e) * P + p;
    }

    // Pencil p and element e that register i holds as an input of a first stage (or an
    // output of a last stage) of radix R; false for registers of idle butterflies.
    template <int R>
    __device__ static __forceinline__ bool pos(int i, int &p, int &e) {
        const int it = i / R, q = i - (i / R) * R;
        const int j = (int)threadIdx.x + it * NT;
        int b;
        decode<R>(j, p, b);
        e = b + q * (L / R);
        return exact(R) || j < items(R);
    }
    template <int DIR>
    __device__ static __forceinline__ bool in_pos(int i, int &p, int &e) { return pos<rad<DIR>(0)>(i, p, e); }
    template <int DIR>
    __device__ static __forceinline__ bool out_pos(int i, int &p, int &e) {
        return pos<rad<DIR>(NSTG - 1)>(i, p, e);
    }

    // Twiddles exp(DIR 2 pi i q k / (NS R)), k = b mod NS, then the radix-R butterflies.
    // tw[m] = exp(-2 pi i m / L).
    template <int DIR, int R, int NS>
    __device__ static __forceinline__ void butterflies(cx<T> *v, const cx<T> *__restrict__ tw) {
#pragma unroll
        for (int it = 0; it < iters(R); ++it) {
            cx<T> *u = v + it * R;
            if constexpr (NS > 1) {
                int p, b;
                decode<R>((int)threadIdx.x + it * NT, p, b);
                const int k = b % NS;
                constexpr int ts = L / (NS * R);
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    cx<T> w = cld(tw + q * k * ts);
                    if (DIR > 0) w.y = -w.y;
                    u[q] = mul(u[q], w);
                }
            }
            bfly<T, DIR, R>(u);
        }
    }

    // In a wave-private tile every stage has radix 4 and one butterfly per thread, so the spans
    // are 1, 4, 16, ... in either direction and a thread's twiddles are the same for every
    // transform of the tile (conjugated for the inverse): they can be loaded once into registers.
    struct Twiddles {
        cx<T> w[NSTG > 1 ? NSTG - 1 : 1][3];
    };
    __device__ static __forceinline__ void load_twiddles(Twiddles &t, const cx<T> *__restrict__ tw) {
        static_assert(WP, "register twiddles need a wave-private tile");
        int p, b;
        decode<4>((int)threadIdx.x, p, b);
#pragma unroll
        for (int s = 1; s < NSTG; ++s) {
            const int NS = 1 << (2 * s);
            const int k = b % NS, ts = L / (NS * 4);
#pragma unroll
            for (int q = 1; q < 4; ++q) t.w[s - 1][q - 1] = cld(tw + q * k * ts);
        }
    }
    template <int DIR, int S>
    __device__ static __forceinline__ void butterflies_reg(cx<T> *v, const Twiddles &t) {
        if constexpr (S > 0) {
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                cx<T> w = t.w[S - 1][q - 1];
                if (DIR > 0) w.y = -w.y;
                v[q] = mul(v[q], w);
            }
        }
        bfly<T, DIR, 4>(v);
    }

    // Any tile: the twiddles of all stages of one direction for this thread's butterflies, loaded
    // once (all in flight together) for the transforms of a block that share that direction.
    template <int DIR>
    static constexpr int tw_count(int upto) {
        int n = 0;
        for (int s = 1; s < upto; ++s) n += iters(rad<DIR>(s)) * (rad<DIR>(s) - 1);
        return n;
    }
    template <int DIR>
    struct TwReg {
        cx<T> w[tw_count<DIR>(NSTG) > 0 ? tw_count<DIR>(NSTG) : 1];
    };
    template <int DIR, int S = 1>
    __device__ static __forceinline__ void load_tw(TwReg<DIR> &t, const cx<T> *__restrict__ tw) {
        if constexpr (S < NSTG) {
            constexpr int R = rad<DIR>(S), NS = span<DIR>(S), ts = L / (NS * R), o = tw_count<DIR>(S);
#pragma unroll
            for (int it = 0; it < iters(R); ++it) {
                int p, b;
                decode<R>((int)threadIdx.x + it * NT, p, b);
                const int k = b % NS;   // idle butterflies read an in-range entry they never use
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    cx<T> w = cld(tw + q * k * ts);
                    if (DIR > 0) w.y = -w.y;
                    t.w[o + it * (R - 1) + q - 1] = w;
                }
            }
            load_tw<DIR, S + 1>(t, tw);
        }
    }
    template <int DIR, int R, int S>
    __device__ static __forceinline__ void butterflies_tw(cx<T> *v, const TwReg<DIR> &t) {
        constexpr int o = tw_count<DIR>(S);
#pragma unroll
        for (int it = 0; it < iters(R); ++it) {
            cx<T> *u = v + it * R;
            if constexpr (S > 0) {
#pragma unroll
                for (int q = 1; q < R; ++q) u[q] = mul(u[q], t.w[o + it * (R - 1) + q - 1]);
            }
            bfly<T, DIR, R>(u);
        }
    }

    // Outputs of a radix-R stage with span NS to the buffer (Stockham order).
    template <int R, int NS>
    __device__ static __forceinline__ void put(const cx<T> *v, cx<T> *buf) {
#pragma unroll
        for (int it = 0; it < iters(R); ++it) {
            const int j = (int)threadIdx.x + it * NT;
            if (!exact(R) && j >= items(R)) continue;
            int p, b;
            decode<R>(j, p, b);
            const int k = b % NS;
            const int o = (b - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[lidx(p, o + q * NS)] = v[it * R + q];
        }
    }
    // Inputs of a radix-R stage from the buffer.
    template <int R>
    __device__ static __forceinline__ void get(cx<T> *v, const cx<T> *buf) {
#pragma unroll
        for (int it = 0; it < iters(R); ++it) {
            const int j = (int)threadIdx.x + it * NT;
            if (!exact(R) && j >= items(R)) continue;
            int p, b;
            decode<R>(j, p, b);
#pragma unroll
            for (int q = 0; q < R; ++q) v[it * R + q] = buf[lidx(p, b + q * (L / R))];
        }
    }

    // The same transform with the twiddles of its direction from registers (any tile).
    template <int DIR, int S = 0>
    __device__ static __forceinline__ void run(cx<T> *v, cx<T> *lds, int &ph, const TwReg<DIR> &t) {
        constexpr int R = rad<DIR>(S), NS = span<DIR>(S);
        butterflies_tw<DIR, R, S>(v, t);
        if constexpr (S + 1 < NSTG) {
            cx<T> *buf = lds;
            if constexpr (NB == 2) {
                buf = lds + (ph ? TILE : 0);
                ph ^= 1;
            } else {
                sync();
            }
            put<R, NS>(v, buf);
            sync();
            get<rad<DIR>(S + 1)>(v, buf);
            run<DIR, S + 1>(v, lds, ph, t);
        }
    }

    // The same transform with the twiddles from registers (wave-private tiles).
    template <int DIR, int S = 0>
    __device__ static __forceinline__ void run(cx<T> *v, cx<T> *lds, int &ph, const Twiddles &t) {
        constexpr int NS = span<DIR>(S);
        butterflies_reg<DIR, S>(v, t);
        if constexpr (S + 1 < NSTG) {
            cx<T> *buf = lds + (ph ? TILE : 0);
            ph ^= 1;
            static_assert(NB == 2, "wave-private tiles alternate two buffers");
            put<4, NS>(v, buf);
            sync();
            get<4>(v, buf);
            run<DIR, S + 1>(v, lds, ph, t);
        }
    }

    // Whole transform (unnormalized; DIR = -1 forward, +1 inverse) of the values in v, which
    // hold the first stage's inputs (in_pos) and end holding the outputs (out_pos).  ph is the
    // caller's buffer phase; it must start at 0 and be passed to every call of the block.
    template <int DIR, int S = 0>
    __device__ static __forceinline__ void run(cx<T> *v, cx<T> *lds, int &ph, const cx<T> *__restrict__ tw) {
        constexpr int R = rad<DIR>(S), NS = span<DIR>(S);
        butterflies<DIR, R, NS>(v, tw);
        if constexpr (S + 1 < NSTG) {
            cx<T> *buf = lds;
            if constexpr (NB == 2) {
                buf = lds + (ph ? TILE : 0);
                ph ^= 1;
            } else {
                sync();
            }
            put<R, NS>(v, buf);
            sync();
            get<rad<DIR>(S + 1)>(v, buf);
            run<DIR, S + 1>(v, lds, ph, tw);
        }
    }
};

// Radix schedules of the lengths with compiled kernels (forward order).
template <int L> struct Plan;
template <> struct Plan<16> { using type = Sched<4, 4>; };
template <> struct Plan<24> { using type = Sched<8, 3>; };
template <> struct Plan<32> { using type = Sched<8, 4>; };
template <> struct Plan<48> { using type = Sched<4, 4, 3>; };
template <> struct Plan<64> { using type = Sched<8, 8>; };
template <> struct Plan<96> { using type = Sched<8, 4, 3>; };
template <> struct Plan<128> { using type = Sched<8, 4, 4>; };
template <> struct Plan<192> { using type = Sched<8, 8, 3>; };
template <> struct Plan<256> { using type = Sched<8, 8, 4>; };
template <> struct Plan<384> { using type = Sched<8, 4, 4, 3>; };
// Schedule of the y and z transforms in precision T: FP64 tiles hold four values per thread,
// so at the power-of-two lengths 64, 128 and 256 radix-4 (and one radix-2) stages keep every
// thread in every stage (a radix-8 stage would leave half of them idle while the other half hold
// eight values).
template <typename T, int L> struct PlanT { using type = typename Plan<L>::type; };
template <> struct PlanT<double, 64> { using type = Sched<4, 4, 4>; };
template <> struct PlanT<double, 128> { using type = Sched<4, 4, 4, 2>; };
template <> struct PlanT<double, 256> { using type = Sched<4, 4, 4, 4>; };

// Schedules of the x passes: radices of at most 4, the first (forward) being 4 and the
// last 4 or 2, so a block of L P / 4 threads holds four values of every pencil-element
// column it owns, the values of several fields at one node stay in one thread, and an
// inverse transform starts from as many registers as it ends with.
template <int L> struct XPlan;
template <> struct XPlan<16> { using type = Sched<4, 4>; };
template <> struct XPlan<24> { using type = Sched<4, 3, 2>; };
template <> struct XPlan<32> { using type = Sched<4, 4, 2>; };
template <> struct XPlan<48> { using type = Sched<4, 3, 4>; };
template <> struct XPlan<64> { using type = Sched<4, 4, 4>; };
template <> struct XPlan<96> { using type = Sched<4, 4, 3, 2>; };
template <> struct XPlan<128> { using type = Sched<4, 4, 4, 2>; };
template <> struct XPlan<192> { using type = Sched<4, 4, 3, 4>; };
template <> struct XPlan<256> { using type = Sched<4, 4, 4, 4>; };
template <> struct XPlan<384> { using type = Sched<4, 4, 4, 3, 2>; };

}  // namespace ct
}  // namespace dft
