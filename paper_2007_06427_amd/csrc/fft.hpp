// Double-precision complex FFT building blocks for gfx950 (CDNA4).
//
// Transforms of length n = 2^p, 8 <= p2 <= 1024, run as a Stockham autosort sequence of
// radix-8 stages, with one radix-2 or radix-4 stage where n is not a power of 8. n/8 threads
// cooperate on one transform. Every thread keeps 8 complex values in registers, and stages
// exchange data through LDS.
//
// Register convention: on entry to and exit from a transform, thread t holds element
// t + m * (n/8) in register slot m, for m = 0 .. 7. Entry and exit positions are the same,
// so an inverse transform can hand its output to a forward transform without touching
// LDS. Pointwise work between the two (products, spectral assembly) runs on registers.
//
// Sign convention: FWD uses exp(-2 pi i), INV uses exp(+2 pi i). Neither scales.
//
// Several transforms share a block. Transform `slot` of `nslot` keeps element e at
// ex[e * nslot + slot], with the slot index fastest, so the lanes of a wavefront touch
// neighbouring 16-byte words.
#pragma once

#include <hip/hip_runtime.h>

namespace lo {

struct cd {
    double x, y;
};

constexpr int TW_N = 4096;  // twiddle table: tw[t] = exp(-2 pi i t / TW_N)

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cd cconj(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.x * s, a.y * s}; }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ cd rot90(cd a) {
    return INV ? cd{-a.y, a.x} : cd{a.y, -a.x};
}

constexpr double kSqrtHalf = 0.70710678118654752440084436210484903928;

// multiply by exp(-+ 2 pi i / 8)
template <bool INV>
__device__ __forceinline__ cd w8_1(cd a) {
    return INV ? cd{(a.x - a.y) * kSqrtHalf, (a.x + a.y) * kSqrtHalf}
               : cd{(a.x + a.y) * kSqrtHalf, (a.y - a.x) * kSqrtHalf};
}
// multiply by exp(-+ 2 pi i 3 / 8)
template <bool INV>
__device__ __forceinline__ cd w8_3(cd a) {
    return INV ? cd{-(a.x + a.y) * kSqrtHalf, (a.x - a.y) * kSqrtHalf}
               : cd{(a.y - a.x) * kSqrtHalf, -(a.x + a.y) * kSqrtHalf};
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
    cd o1 = w8_1<INV>(x3), o2 = rot90<INV>(x5), o3 = w8_3<INV>(x7);
    cd e0 = x0, e1 = x2, e2 = x4, e3 = x6, o0 = x1;
    x0 = cadd(e0, o0);
    x4 = csub(e0, o0);
    x1 = cadd(e1, o1);
    x5 = csub(e1, o1);
    x2 = cadd(e2, o2);
    x6 = csub(e2, o2);
    x3 = cadd(e3, o3);
    x7 = csub(e3, o3);
}

// Radix plan per length: radix-8 stages, with one radix-2/4 stage last where needed.
template <int N>
struct Plan;
template <> struct Plan<8>    { static constexpr int S = 1; static constexpr int R[4] = {8, 0, 0, 0}; };
template <> struct Plan<16>   { static constexpr int S = 2; static constexpr int R[4] = {8, 2, 0, 0}; };
template <> struct Plan<32>   { static constexpr int S = 2; static constexpr int R[4] = {8, 4, 0, 0}; };
template <> struct Plan<64>   { static constexpr int S = 2; static constexpr int R[4] = {8, 8, 0, 0}; };
template <> struct Plan<128>  { static constexpr int S = 3; static constexpr int R[4] = {8, 8, 2, 0}; };
template <> struct Plan<256>  { static constexpr int S = 3; static constexpr int R[4] = {8, 8, 4, 0}; };
template <> struct Plan<512>  { static constexpr int S = 3; static constexpr int R[4] = {8, 8, 8, 0}; };
template <> struct Plan<1024> { static constexpr int S = 4; static constexpr int R[4] = {8, 8, 8, 2}; };

template <bool INV>
__device__ __forceinline__ cd twiddle(const cd* __restrict__ tw, int idx) {
    cd w = tw[idx];
    return INV ? cconj(w) : w;
}

// One Stockham stage: radix R, span NS (product of earlier radices), for thread t.
// Butterfly i of the thread is b = t + i * (N/8); its element r lives in slot i + r * (8/R).
template <int N, int R, int NS, bool INV>
__device__ __forceinline__ void compute_stage(cd v[8], int t, const cd* __restrict__ tw) {
    constexpr int NB = 8 / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * (N / 8);
        if constexpr (NS > 1) {
            const int k = b % NS;
            constexpr int step = TW_N / (NS * R);
#pragma unroll
            for (int r = 1; r < R; ++r) v[i + r * NB] = cmul(v[i + r * NB], twiddle<INV>(tw, k * r * step));
        }
        if constexpr (R == 8) {
            dft8<INV>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
        } else if constexpr (R == 4) {
            dft4<INV>(v[i], v[i + 2], v[i + 4], v[i + 6]);
        } else {
            dft2<INV>(v[i], v[i + 4]);
        }
    }
}

// Scatter the outputs of a stage (radix R, span NS) to LDS.
template <int N, int R, int NS>
__device__ __forceinline__ void write_stage_outputs(const cd v[8], int t, cd* ex, int nslot) {
    constexpr int NB = 8 / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * (N / 8);
        const int base = (b / NS) * NS * R + (b % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) ex[(base + r * NS) * nslot] = v[i + r * NB];
    }
}

// Gather the inputs of a stage of radix R from LDS.
template <int N, int R>
__device__ __forceinline__ void read_stage_inputs(cd v[8], int t, const cd* ex, int nslot) {
    constexpr int NB = 8 / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * (N / 8);
#pragma unroll
        for (int r = 0; r < R; ++r) v[i + r * NB] = ex[(b + r * (N / R)) * nslot];
    }
}

template <int N, bool INV, int S, int NS>
__device__ __forceinline__ void run_stages(cd v[8], int t, cd* ex, int nslot, const cd* __restrict__ tw) {
    constexpr int R = Plan<N>::R[S];
    if constexpr (S > 0) {
        constexpr int Rp = Plan<N>::R[S - 1];
        write_stage_outputs<N, Rp, NS / Rp>(v, t, ex, nslot);
        __syncthreads();
        read_stage_inputs<N, R>(v, t, ex, nslot);
        __syncthreads();
    }
    compute_stage<N, R, NS, INV>(v, t, tw);
    if constexpr (S + 1 < Plan<N>::S) run_stages<N, INV, S + 1, NS * R>(v, t, ex, nslot, tw);
}

// Full length-N transform of the values in v (see the register convention above).
// ex points at this transform's slot in the shared exchange buffer; every thread of the
// block must call this (it contains block barriers when N > 8).
template <int N, bool INV>
__device__ __forceinline__ void fft(cd v[8], int t, cd* ex, int nslot, const cd* __restrict__ tw) {
    run_stages<N, INV, 0, 1>(v, t, ex, nslot, tw);
}

}  // namespace lo
