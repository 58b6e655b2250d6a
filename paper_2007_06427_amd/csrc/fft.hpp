// Double-precision complex FFT building blocks for gfx950 (CDNA4).
//
// A transform of length n = 2^p (8 <= n <= 1024) runs as a Stockham autosort sequence of
// radix-2/4/8/16 stages on PT points per thread (PT = 8 or 16), n/PT threads per transform.
// When n/PT <= 64 the transform lives inside one wavefront: stages exchange data through
// that wavefront's own LDS region and need no block barrier. Longer transforms span several
// wavefronts and synchronise with block barriers.
//
// Register convention: on entry to and exit from a transform, thread t of the transform
// holds element t + m * (n/PT) in register slot m, for m = 0 .. PT-1. Entry and exit
// positions are the same, so an inverse transform can hand its output to a forward
// transform in registers. Pointwise work between the two (products, spectral assembly)
// touches no memory.
//
// Sign convention: FWD uses exp(-2 pi i), INV uses exp(+2 pi i). Neither scales.
//
// LDS exchange: a transform's region holds n + n/8 complex values. Element `pos` sits at
// pos + pos/8: one 16-byte pad every 8 elements, which makes the stride-8 and stride-16
// scatters of the early stages free of bank conflicts on 64 banks of 4 bytes.
#pragma once

#include <hip/hip_runtime.h>

namespace lo {

struct cd {
    double x, y;
};

constexpr int TW_N = 4096;  // twiddle table: tw[t] = exp(-2 pi i t / TW_N)

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
// Complex product with two fused multiply-adds (explicit, so every kernel that inlines it
// rounds it the same way).
__device__ __forceinline__ cd cmul(cd a, cd b) {
    return {__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ cd cconj(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.x * s, a.y * s}; }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ cd rot90(cd a) {
    return INV ? cd{-a.y, a.x} : cd{a.y, -a.x};
}

constexpr double kSqrtHalf = 0.70710678118654752440084436210484903928;
constexpr double kCos8 = 0.92387953251128675612818318939678828682;  // cos(pi/8)
constexpr double kSin8 = 0.38268343236508977172845998403039886676;  // sin(pi/8)

// multiply by exp(-+ 2 pi i m / 16) for a compile-time m
template <bool INV, int m>
__device__ __forceinline__ cd w16(cd a) {
    constexpr int mm = m % 16;
    if constexpr (mm == 0) {
        return a;
    } else if constexpr (mm == 4) {
        return rot90<INV>(a);
    } else if constexpr (mm == 8) {
        return cd{-a.x, -a.y};
    } else if constexpr (mm == 12) {
        return rot90<!INV>(a);
    } else if constexpr (mm % 4 == 2) {
        // odd multiples of pi/4: (x, y) (c, sy) with |c| = |sy| = sqrt(1/2), one add and one
        // product per component
        constexpr double c = (mm == 2 || mm == 14) ? kSqrtHalf : -kSqrtHalf;
        constexpr double sy = ((mm == 2 || mm == 6) ? kSqrtHalf : -kSqrtHalf) * (INV ? 1.0 : -1.0);
        if constexpr (c == sy) {
            return cd{(a.x - a.y) * c, (a.x + a.y) * c};
        } else {
            return cd{(a.x + a.y) * c, (a.y - a.x) * c};
        }
    } else {
        // cos and sin of 2 pi mm / 16 from the first-octant constants
        constexpr double c = (mm == 1 || mm == 15) ? kCos8 : (mm == 2 || mm == 14) ? kSqrtHalf
                           : (mm == 3 || mm == 13) ? kSin8 : (mm == 5 || mm == 11) ? -kSin8
                           : (mm == 6 || mm == 10) ? -kSqrtHalf : -kCos8;  // 7, 9
        constexpr double s = (mm == 1 || mm == 7) ? kSin8 : (mm == 2 || mm == 6) ? kSqrtHalf
                           : (mm == 3 || mm == 5) ? kCos8 : (mm == 9 || mm == 15) ? -kSin8
                           : (mm == 10 || mm == 14) ? -kSqrtHalf : -kCos8;  // 11, 13
        // forward: exp(-i theta) = (c, -s); inverse: (c, s)
        constexpr double sy = INV ? s : -s;
        return cd{__builtin_fma(a.x, c, -(a.y * sy)), __builtin_fma(a.x, sy, a.y * c)};
    }
}

template <bool INV>
__device__ __forceinline__ void dft2(cd& a, cd& b) {
    cd t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(cd& x0, cd& x1, cd& x2, cd& x3) {
    cd t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = rot90<INV>(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(cd& x0, cd& x1, cd& x2, cd& x3, cd& x4, cd& x5, cd& x6, cd& x7) {
    // radix-2 split over even and odd inputs, each a length-4 DFT
    dft4<INV>(x0, x2, x4, x6);  // E0..E3
    dft4<INV>(x1, x3, x5, x7);  // O0..O3
    const cd o1 = w16<INV, 2>(x3), o2 = w16<INV, 4>(x5), o3 = w16<INV, 6>(x7);
    const cd e0 = x0, e1 = x2, e2 = x4, e3 = x6, o0 = x1;
    x0 = cadd(e0, o0);
    x4 = csub(e0, o0);
    x1 = cadd(e1, o1);
    x5 = csub(e1, o1);
    x2 = cadd(e2, o2);
    x6 = csub(e2, o2);
    x3 = cadd(e3, o3);
    x7 = csub(e3, o3);
}

// 16-point DFT of v[s0 + r * st], r = 0..15 (natural order in and out), as 4 x 4:
// inputs n = 4 n1 + n2, outputs k = k1 + 4 k2.
template <bool INV, int st>
__device__ __forceinline__ void dft16(cd* v, int s0) {
    cd y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cd a = v[s0 + (0 + n2) * st], b = v[s0 + (4 + n2) * st], c = v[s0 + (8 + n2) * st],
           d = v[s0 + (12 + n2) * st];
        dft4<INV>(a, b, c, d);  // over n1: outputs k1 = 0..3
        y[n2 * 4 + 0] = a;
        y[n2 * 4 + 1] = b;
        y[n2 * 4 + 2] = c;
        y[n2 * 4 + 3] = d;
    }
    // twiddle W16^(n2 k1)
    y[1 * 4 + 1] = w16<INV, 1>(y[1 * 4 + 1]);
    y[1 * 4 + 2] = w16<INV, 2>(y[1 * 4 + 2]);
    y[1 * 4 + 3] = w16<INV, 3>(y[1 * 4 + 3]);
    y[2 * 4 + 1] = w16<INV, 2>(y[2 * 4 + 1]);
    y[2 * 4 + 2] = w16<INV, 4>(y[2 * 4 + 2]);
    y[2 * 4 + 3] = w16<INV, 6>(y[2 * 4 + 3]);
    y[3 * 4 + 1] = w16<INV, 3>(y[3 * 4 + 1]);
    y[3 * 4 + 2] = w16<INV, 6>(y[3 * 4 + 2]);
    y[3 * 4 + 3] = w16<INV, 9>(y[3 * 4 + 3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cd a = y[0 * 4 + k1], b = y[1 * 4 + k1], c = y[2 * 4 + k1], d = y[3 * 4 + k1];
        dft4<INV>(a, b, c, d);  // over n2: outputs k2 = 0..3
        v[s0 + (k1 + 0) * st] = a;
        v[s0 + (k1 + 4) * st] = b;
        v[s0 + (k1 + 8) * st] = c;
        v[s0 + (k1 + 12) * st] = d;
    }
}

// Radix plan per length and points per thread (product = N, every radix divides PT).
template <int N, int PT>
struct Plan;
template <> struct Plan<8, 8>     { static constexpr int S = 1; static constexpr int R[4] = {8, 0, 0, 0}; };
template <> struct Plan<16, 8>    { static constexpr int S = 2; static constexpr int R[4] = {8, 2, 0, 0}; };
template <> struct Plan<32, 8>    { static constexpr int S = 2; static constexpr int R[4] = {8, 4, 0, 0}; };
template <> struct Plan<64, 8>    { static constexpr int S = 2; static constexpr int R[4] = {8, 8, 0, 0}; };
template <> struct Plan<128, 8>   { static constexpr int S = 3; static constexpr int R[4] = {8, 8, 2, 0}; };
template <> struct Plan<256, 8>   { static constexpr int S = 3; static constexpr int R[4] = {8, 8, 4, 0}; };
template <> struct Plan<512, 8>   { static constexpr int S = 3; static constexpr int R[4] = {8, 8, 8, 0}; };
template <> struct Plan<1024, 8>  { static constexpr int S = 4; static constexpr int R[4] = {8, 8, 8, 2}; };
template <> struct Plan<1024, 16> { static constexpr int S = 3; static constexpr int R[4] = {16, 8, 8, 0}; };
// Four points per thread (short row transforms spread over more threads).
template <> struct Plan<8, 4>     { static constexpr int S = 2; static constexpr int R[4] = {4, 2, 0, 0}; };
template <> struct Plan<16, 4>    { static constexpr int S = 2; static constexpr int R[4] = {4, 4, 0, 0}; };
template <> struct Plan<32, 4>    { static constexpr int S = 3; static constexpr int R[4] = {4, 4, 2, 0}; };
template <> struct Plan<64, 4>    { static constexpr int S = 3; static constexpr int R[4] = {4, 4, 4, 0}; };

template <int N>
constexpr int xlen() {  // padded exchange length
    return N + N / 8;
}
__device__ __forceinline__ int xpos(int pos) { return pos + (pos >> 3); }

// Per-thread twiddle cache. In stage s (radix R, span NS) butterfly i of thread t needs
// w^(k r), r = 1 .. R-1, with w = exp(-2 pi i / (NS R)) and k = (t + i N/PT) mod NS. These
// depend only on t, so a thread loads them once and reuses them for every transform it runs.
// Per butterfly the cache holds w^k, w^2k, w^4k (and w^8k for radix 16) as read from the
// table, and the other powers are formed by one or two complex products: w^3k =
// w^k w^2k, w^5k = w^k w^4k, w^6k = w^2k w^4k, w^7k = w^3k w^4k, and for radix 16
// w^(8k + m) = w^8k w^(mk). Each twiddle is within a few units in the last place. The
// inverse transform uses the conjugates.
template <int N, int PT>
struct TwCache {
    static constexpr int NBASE = 4;                  // base powers kept per butterfly
    static constexpr int MAXNB = PT / 2;             // butterflies per thread in a radix-2 stage
    cd w[4][MAXNB][NBASE];                           // [stage][butterfly][1, 2, 4, 8]
};

template <int N, int PT, int S, int NS>
__device__ __forceinline__ void tw_cache_fill(TwCache<N, PT>& c, int t, const cd* __restrict__ tw) {
    constexpr int R = Plan<N, PT>::R[S];
    if constexpr (NS > 1) {
        constexpr int NB = PT / R;
        constexpr int step = TW_N / (NS * R);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int k = (t + i * (N / PT)) % NS;
            c.w[S][i][0] = tw[(k * step) & (TW_N - 1)];
            if constexpr (R >= 4) c.w[S][i][1] = tw[(2 * k * step) & (TW_N - 1)];
            if constexpr (R >= 8) c.w[S][i][2] = tw[(4 * k * step) & (TW_N - 1)];
            if constexpr (R >= 16) c.w[S][i][3] = tw[(8 * k * step) & (TW_N - 1)];
        }
    }
    if constexpr (S + 1 < Plan<N, PT>::S) tw_cache_fill<N, PT, S + 1, NS * R>(c, t, tw);
}

template <int N, int PT>
__device__ __forceinline__ void tw_cache_load(TwCache<N, PT>& c, int t, const cd* __restrict__ tw) {
    tw_cache_fill<N, PT, 0, 1>(c, t, tw);
}

// An opaque copy of a cached twiddle: products formed from it are not merged with products
// formed for another transform, so the derived powers do not stay live between transforms.
__device__ __forceinline__ cd opaque(cd w) {
    asm volatile("" : "+v"(w.x), "+v"(w.y));
    return w;
}

template <bool INV>
__device__ __forceinline__ cd cmul_tw(cd a, cd w) {
    return INV ? cd{__builtin_fma(a.x, w.x, a.y * w.y), __builtin_fma(a.y, w.x, -(a.x * w.y))} : cmul(a, w);
}

// Apply w^(k r) to element r of butterfly i (elements in slots i + r NB), from the cache.
template <int R, int NB, bool INV>
__device__ __forceinline__ void apply_twiddles(cd* v, int i, const cd* base) {
    const cd w1 = opaque(base[0]);
    v[i + NB] = cmul_tw<INV>(v[i + NB], w1);
    if constexpr (R >= 4) {
        const cd w2 = opaque(base[1]);
        const cd w3 = cmul(w1, w2);
        v[i + 2 * NB] = cmul_tw<INV>(v[i + 2 * NB], w2);
        v[i + 3 * NB] = cmul_tw<INV>(v[i + 3 * NB], w3);
        if constexpr (R >= 8) {
            const cd w4 = opaque(base[2]);
            v[i + 4 * NB] = cmul_tw<INV>(v[i + 4 * NB], w4);
            v[i + 5 * NB] = cmul_tw<INV>(v[i + 5 * NB], cmul(w1, w4));
            v[i + 6 * NB] = cmul_tw<INV>(v[i + 6 * NB], cmul(w2, w4));
            v[i + 7 * NB] = cmul_tw<INV>(v[i + 7 * NB], cmul(w3, w4));
            if constexpr (R >= 16) {
                const cd w8 = opaque(base[3]);
                v[i + 8 * NB] = cmul_tw<INV>(v[i + 8 * NB], w8);
#pragma unroll
                for (int m = 1; m < 8; ++m) {
                    const cd wm = (m == 1) ? w1 : (m == 2) ? w2 : (m == 3) ? w3 : (m == 4) ? w4
                                : (m == 5) ? cmul(w1, w4) : (m == 6) ? cmul(w2, w4) : cmul(w3, w4);
                    v[i + (8 + m) * NB] = cmul_tw<INV>(v[i + (8 + m) * NB], cmul(w8, wm));
                }
            }
        }
    }
}

// Wavefront-level LDS ordering. The LDS performs the operations of one wavefront in the order
// they were issued, so a read issued after a write of the same wavefront returns what the
// write stored, for every lane, without waiting for the write to complete (a wait is needed
// only between wavefronts). Only the compiler has to keep the order: no memory operation
// moves across this point. Read results are waited for where they are used.
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

// Ordering between stages: wavefront order when the transform fits in one wavefront,
// otherwise a block barrier (every thread of the block then runs the same transform code).
template <int TPF>
__device__ __forceinline__ void xsync() {
    if constexpr (TPF <= 64) {
        wave_lds_order();
    } else {
        __syncthreads();
    }
}

// One Stockham stage: radix R, span NS (product of earlier radices), for thread t.
// Butterfly i of the thread is b = t + i * (N/PT); its element r lives in slot i + r * (PT/R).
template <int N, int PT, int S, int R, int NS, bool INV>
__device__ __forceinline__ void compute_stage(cd* v, const TwCache<N, PT>& c) {
    constexpr int NB = PT / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if constexpr (NS > 1) apply_twiddles<R, NB, INV>(v, i, c.w[S][i]);
        if constexpr (R == 16) {
            dft16<INV, NB>(v, i);
        } else if constexpr (R == 8) {
            dft8<INV>(v[i], v[i + NB], v[i + 2 * NB], v[i + 3 * NB], v[i + 4 * NB], v[i + 5 * NB], v[i + 6 * NB],
                      v[i + 7 * NB]);
        } else if constexpr (R == 4) {
            dft4<INV>(v[i], v[i + NB], v[i + 2 * NB], v[i + 3 * NB]);
        } else {
            dft2<INV>(v[i], v[i + NB]);
        }
    }
}

template <int N, int PT, int R, int NS>
__device__ __forceinline__ void write_stage_outputs(const cd* v, int t, cd* ex) {
    constexpr int NB = PT / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * (N / PT);
        const int base = (b / NS) * NS * R + (b % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) ex[xpos(base + r * NS)] = v[i + r * NB];
    }
}

template <int N, int PT, int R>
__device__ __forceinline__ void read_stage_inputs(cd* v, int t, const cd* ex) {
    constexpr int NB = PT / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * (N / PT);
#pragma unroll
        for (int r = 0; r < R; ++r) v[i + r * NB] = ex[xpos(b + r * (N / R))];
    }
}

template <int N, int PT, bool INV, int S, int NS>
__device__ __forceinline__ void run_stages(cd* v, int t, cd* ex, const TwCache<N, PT>& c) {
    constexpr int R = Plan<N, PT>::R[S];
    if constexpr (S > 0) {
        constexpr int Rp = Plan<N, PT>::R[S - 1];
        write_stage_outputs<N, PT, Rp, NS / Rp>(v, t, ex);
        xsync<N / PT>();
        read_stage_inputs<N, PT, R>(v, t, ex);
        xsync<N / PT>();
    }
    compute_stage<N, PT, S, R, NS, INV>(v, c);
    if constexpr (S + 1 < Plan<N, PT>::S) run_stages<N, PT, INV, S + 1, NS * R>(v, t, ex, c);
}

// Full length-N transform of the values in v (see the register convention above). All
// threads of the transform must be in the calling wavefront; ex is the transform's own
// exchange region of xlen<N>() values.
template <int N, int PT, bool INV>
__device__ __forceinline__ void fft(cd* v, int t, cd* ex, const TwCache<N, PT>& c) {
    run_stages<N, PT, INV, 0, 1>(v, t, ex, c);
}

}  // namespace lo
