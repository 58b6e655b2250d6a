// LDS-resident form of the fictitious-time step (Sec. 4.2): one block holds one loop's band
// state and its two live intermediates in LDS and runs every pass of every step in one
// launch, so HBM sees only the state's load and store. It applies where a loop's working
// set fits in the 160 KB of LDS of a CU (for example 32 x 256, 64 x 128, 128 x 64).
//
// The column passes are the HBM form's own pass bodies (col_pass_A/C/E) pointed at LDS
// arrays. The row passes are restated here to read and write the resident arrays directly
// instead of staging tiles, with the same row pairing, transforms, products and split, and
// the per-loop sums use the same fixed order. A step therefore gives the same bits as the
// HBM form.
//
// LDS carve (complex values unless noted), for a loop of M x N (Nx x Ns):
//   U  [C][NB]   band state; pass C overwrites it with U1 = u + dtau sigma G_lin, pass E
//                with the new state (each element is read before it is written, by one thread)
//   A  [C][N]    u after the inverse s-transforms (pass A, or E fused with the next A)
//   X  [C][N]    B, then C (in place, column by column), then D (in place, pair by pair)
//   EX           exchange regions: ColG<N>::LDS for the column passes, or one region of
//                xlen<M>() + 1 values per pair of rows for the row passes
//   2C doubles   per-column partial sums of J and dJ/dT
//   12 doubles   T, T_old, J, dJ/dT and the two-wavefront reduction slots
#pragma once

#include "passes.hpp"

namespace lo {

// Exchange stride of one pair of rows in the resident row passes.
template <int M>
constexpr int res_rxs() {
    return xlen<M>() + 1;
}

template <int M, int N>
struct ResG {
    static constexpr int C = (M - 1) / 3 + 1;
    static constexpr int Ks = (N - 1) / 3;
    static constexpr int NB = 2 * Ks + 1;
    static constexpr int W = C * N;
    static constexpr int S = C * NB;
    // Row pass lanes are mapped pair-fastest within a wavefront, so consecutive lanes touch
    // consecutive rows of A and X; an odd exchange stride keeps their regions on distinct banks.
    static constexpr int RX = RowG<M>::P * res_rxs<M>();
    static constexpr int EX = ColG<N>::LDS > RX ? ColG<N>::LDS : RX;
    static constexpr int DOUBLES = 2 * C + 12;
    static constexpr size_t BYTES = sizeof(cd) * (size_t)(S + 2 * W + EX) + sizeof(double) * DOUBLES;
    static constexpr bool FITS = BYTES <= 160 * 1024 && N <= 512 && M <= 128;
    // Two blocks share a CU where both fit its LDS; the kernel is then compiled for two
    // wavefronts per SIMD (at most 256 registers each, a few spilled), which costs a lone
    // block 5-8% but lets a second loop hide the first one's latency.
    static constexpr int BLOCKS_PER_CU = BYTES <= 80 * 1024 ? 2 : 1;
    static constexpr int COL_ROUNDS = (C + ColG<N>::F - 1) / ColG<N>::F;
    static constexpr int ROW_ROUNDS = (N + RowG<M>::ROWS - 1) / RowG<M>::ROWS;
};

// Thread roles in a resident row pass: transform group p (pair of rows), lane t in it.
template <int M>
struct ResRowLane {
    int t, p;
    __device__ ResRowLane() {
        constexpr int TPF = RowG<M>::TPF, PW = 64 / TPF;
        const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
        t = lane / PW;
        p = wave * PW + lane % PW;
    }
};

// Element e of the Hermitian extension of row r of a resident [j][n] array (zero for rows
// past the loop, as the HBM form's tiles hold for them).
__device__ __forceinline__ cd res_herm(const cd* X, int N, int r, bool ok, int e, int M, int Kx) {
    return ok ? herm_ext(X, N, r, e, M, Kx) : cd{0.0, 0.0};
}

// Products of the pair's two fields, forward transform and split (the same arithmetic as
// row_products), written to rows a and b of X.
template <int M>
__device__ __forceinline__ void res_row_products(const Shape& sh, cd* va, cd* vb, cd* ex, int t, cd* X, int a,
                                                 int b, bool oka, bool okb, const TwCache<M, RowG<M>::PT>& twc) {
    using G = RowG<M>;
    fft<M, G::PT, true>(va, t, ex, twc);
    fft<M, G::PT, true>(vb, t, ex, twc);
#pragma unroll
    for (int m = 0; m < G::PT; ++m) va[m] = cd{va[m].x * vb[m].x, va[m].y * vb[m].y};
    fft<M, G::PT, false>(va, t, ex, twc);
#pragma unroll
    for (int m = 0; m < G::PT; ++m) ex[xpos(t + m * G::TPF)] = va[m];
    wave_lds_order();
    const double s = 0.5 / M;
    for (int j = t; j < sh.C; j += G::TPF) {
        const cd za = ex[xpos(j)];
        const cd zb = ex[xpos((M - j) & (M - 1))];
        if (oka) X[j * sh.N + a] = cd{(za.x + zb.x) * s, (za.y - zb.y) * s};
        if (okb) X[j * sh.N + b] = cd{(za.y + zb.y) * s, (zb.x - za.x) * s};
    }
    wave_lds_order();  // the exchange region is reused by this group's next transform
}

// Pass B for the pairs of row tile `tile`: X = (u u_x) = (1/2) (u^2)_x per row, from A (the
// same arithmetic as row_square_dx; resident rows are never longer than kSquareMaxM).
template <int M>
__device__ __forceinline__ void res_row_B(const Shape& sh, int tile, const cd* A, cd* X, cd* exr,
                                          const cd* __restrict__ tw) {
    using G = RowG<M>;
    static_assert(M <= kSquareMaxM, "the resident form takes the square form of u u_x");
    const ResRowLane<M> ln;
    const int a = tile * G::ROWS + ln.p, b = a + G::P;
    const bool oka = a < sh.N, okb = b < sh.N;
    TwCache<M, G::PT> twc;
    tw_cache_load<M, G::PT>(twc, ln.t, tw);
    cd va[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = ln.t + m * G::TPF;
        va[m] = pack2(res_herm(A, sh.N, a, oka, e, M, sh.Kx), res_herm(A, sh.N, b, okb, e, M, sh.Kx));
    }
    cd* ex = exr + ln.p * res_rxs<M>();
    fft<M, G::PT, true>(va, ln.t, ex, twc);
#pragma unroll
    for (int m = 0; m < G::PT; ++m) va[m] = cd{va[m].x * va[m].x, va[m].y * va[m].y};
    fft<M, G::PT, false>(va, ln.t, ex, twc);
#pragma unroll
    for (int m = 0; m < G::PT; ++m) ex[xpos(ln.t + m * G::TPF)] = va[m];
    wave_lds_order();
    const double hq = (kTwoPi / sh.L) * (0.25 / M);
    for (int j = ln.t; j < sh.C; j += G::TPF) {
        const cd za = ex[xpos(j)];
        const cd zb = ex[xpos((M - j) & (M - 1))];
        const double c = hq * j;
        if (oka) X[j * sh.N + a] = cd{c * (zb.y - za.y), c * (za.x + zb.x)};
        if (okb) X[j * sh.N + b] = cd{c * (za.x - zb.x), c * (za.y + zb.y)};
    }
    wave_lds_order();  // the exchange region is reused by this group's next transform
}

// Pass D for the pairs of row tile `tile`: X = (u r_x) per row, from A and X (r_x), in place.
template <int M>
__device__ __forceinline__ void res_row_D(const Shape& sh, int tile, const cd* A, cd* X, cd* exr,
                                          const cd* __restrict__ tw) {
    using G = RowG<M>;
    const ResRowLane<M> ln;
    const int a = tile * G::ROWS + ln.p, b = a + G::P;
    const bool oka = a < sh.N, okb = b < sh.N;
    TwCache<M, G::PT> twc;
    tw_cache_load<M, G::PT>(twc, ln.t, tw);
    cd va[G::PT], vb[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = ln.t + m * G::TPF;
        va[m] = pack2(res_herm(A, sh.N, a, oka, e, M, sh.Kx), res_herm(A, sh.N, b, okb, e, M, sh.Kx));
        vb[m] = pack2(res_herm(X, sh.N, a, oka, e, M, sh.Kx), res_herm(X, sh.N, b, okb, e, M, sh.Kx));
    }
    // every read of rows a and b of X (by this group only) precedes the group's writes below
    res_row_products<M>(sh, va, vb, exr + ln.p * res_rxs<M>(), ln.t, X, a, b, oka, okb, twc);
}

}  // namespace lo
