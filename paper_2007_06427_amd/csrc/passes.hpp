// The passes of one fictitious-time step of the KS loop dynamics, as block-level device
// functions over one tile of a batch of loops (Sec. 4.2 of Azimi, Ashtari & Schneider,
// arXiv:2007.06427).
//
// Notation: M = Nx and N = Ns grid points. The band is |j| <= Kx and |k| <= Ks, with
// Kx = (M-1)/3 and Ks = (N-1)/3. C = Kx + 1 retained non-negative spatial modes and
// NB = 2 Ks + 1 retained temporal modes. q_j = 2 pi j / L and omega_k = 2 pi k.
//
// Pass A (columns): A(j, s_n) = sum_k u_hat_{j,k} e^{2 pi i n k / N}, an inverse
//                   s-transform of each retained column.
// Pass B (rows):    u at (x_m, s_n) from the inverse x-transform of A(., s_n); u^2 on the
//                   grid; B(j, s_n) = (i q_j / 2) times the forward x-transform of u^2, j < C,
//                   which is the transform of u u_x = (1/2) (u^2)_x. Rows longer than
//                   kSquareMaxM take u_x from a second inverse transform and the product u u_x
//                   instead (accuracy, see kSquareMaxM). (Each transform carries two rows.)
// Pass C (columns): w_hat = forward s-transform of B, then the residual of eq. KS_R,
//                     r_hat = -(i omega/T) u_hat - w_hat + q^2 u_hat - q^4 u_hat.
//                   Per-column partial sums of J and dJ/dT. The linear part of the flow,
//                     G_lin = (-i omega/T - q^2 + q^4) r_hat,
//                   stored as G_lin itself, or, when stepping, folded into the update as
//                     U1 = u_hat + dtau sigma G_lin.
//                   C(j, s_n) = inverse s-transform of i q r_hat (r_x by columns).
// Pass D (rows):    u and r_x at each row, p = u r_x, D(j, s_n) = forward x-transform of p.
//                   The block holding row 0 of a loop finishes J and dJ/dT (and T's update).
// Pass E (columns): p_hat = forward s-transform of D, so G_1 = G_lin - p_hat (eq. KS_G),
//                   or u_hat' = U1 - dtau sigma p_hat when stepping. Optionally it also
//                   runs pass A of the next step on the new column, while it is still in
//                   registers.
//
// u u_x is formed as (1/2) (u^2)_x on rows of up to kSquareMaxM points (the square in physical
// space, the paper's pseudo-spectral treatment of products, and the derivative in spectral
// space) and as the product u * u_x on longer rows; u r_x is always a product in physical space.
// Every product is of band-limited fields on the full grid, so it is free of aliasing inside
// the band, and differentiating the square there is exact. Truncation to the band is implicit:
// only retained modes are ever formed.
//
// Device layouts (complex values, interleaved doubles), one loop after another:
//   band state U, G   [l][j][kk]  j < C, kk < NB: kk = k (k >= 0), kk = k + NB (k < 0)
//   intermediates     [l][j][n]   j < C, n < N
// Columns are contiguous, so column passes read and write whole columns. Row passes stage
// a tile of rows through LDS.
#pragma once

#include "fft.hpp"

namespace lo {

constexpr int kBlock = 256;  // threads per block for every pass kernel

enum Mode : int {
    MODE_RESIDUAL = 0,  // pass C writes r_hat (band layout) into G
    MODE_COST = 1,      // pass C partials only
    MODE_GRAD = 2,      // pass C writes G_lin, pass E turns it into G_1
    MODE_STEP = 3,      // pass C writes U1, pass D advances T, pass E writes u_hat'
    MODE_ADJOINT = 4,   // reverse mode from a saved residual: pass D skips the finalize, pass E
                        // forms G_lin from R and writes scale_l w_j G_1 into G
};

struct Shape {
    int M, N;    // grid points in x and s
    int Kx, Ks;  // band limits
    int H;       // M/2 + 1 columns of the rfft layout
    int C;       // Kx + 1 retained columns
    int NB;      // 2 Ks + 1 retained temporal modes
    int logN;    // log2(N)
    int nloops;
    double L;
};

struct Work {
    cd* A;            // [l][j][n]
    cd* BD;           // [l][j][n]   (B, then D)
    cd* Cb;           // [l][j][n]
    cd* U;            // [l][j][kk]  band state
    cd* G;            // [l][j][kk]  G_lin, U1, r_hat or G_1 depending on the mode
    double* partial;  // [l][j][2]   per-column sums: w_j |r|^2 and w_j Re(u_s conj r)
    double* J;        // [l]
    double* dJdT;     // [l]
    double* Told;     // [l]  period at the start of the current step
    int* status;      // sticky device status
    const cd* R;      // [l][j][kk] saved residual r_hat (MODE_ADJOINT)
    const double* gJ;  // [l] cotangent of J (MODE_ADJOINT; null: all ones)
    const double* dJdT_in;  // [l] dJ/dT of the forward (MODE_ADJOINT)
    double* grad_T;   // [l] gJ dJ/dT, written by pass E (MODE_ADJOINT; null: skipped)
    int herm0;        // U is caller-owned: read column 0 through its Hermitian part
};

// Band index of the temporal partner -k of band index kk (k -> -k).
__device__ __forceinline__ int band_partner(int kk, int NB) { return kk == 0 ? 0 : NB - kk; }

// Band value u[kk] of column j; with herm0, column 0 is read through its Hermitian part
// (u_{0,k} + conj u_{0,-k}) / 2, the part a real field keeps.
__device__ __forceinline__ cd band_get(const cd* u, int j, int kk, int NB, int herm0) {
    const cd v = u[kk];
    if (herm0 && j == 0) {
        const cd w = u[band_partner(kk, NB)];
        return cd{0.5 * (v.x + w.x), 0.5 * (v.y - w.y)};
    }
    return v;
}

constexpr double kTwoPi = 6.283185307179586476925286766559005768;

// compact band index of FFT-order row e, or -1 outside the band
__device__ __forceinline__ int band_row(int e, int N, int Ks) {
    if (e <= Ks) return e;
    if (e >= N - Ks) return e - (N - 2 * Ks - 1);
    return -1;
}

__device__ __forceinline__ double wsum_lanes(double x, int width) {
    // sum over aligned groups of `width` lanes (a power of two <= 64), fixed xor-tree order
    for (int o = width / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// ---------------------------------------------------------------------------- column passes
// TPF = N/PT threads per column transform, F = kBlock / TPF columns per block, thread
// tid -> t = tid % TPF (position within the transform), f = tid / TPF (column in block).
// Column c = block * F + f runs over nloops * C columns, loop-major. Every column length takes
// 8 points per thread: a 1024-point column spans two wavefronts (radix 8, 8, 8, 2, block
// barriers between stages). 16 points per thread, one wavefront per column and two exchanges,
// measured slower on 64 loops of 256 x 1024 (pass C 57.8 against 52.8 us, the reverse pass's
// column pass 79.9 against 73.9 us): the LDS of a column is the same, so a CU holds the same
// columns, on half the wavefronts.
__host__ __device__ constexpr int col_pt(int) { return 8; }
__host__ __device__ constexpr int col_per_block(int N) { return kBlock / (N / col_pt(N)); }

template <int N>
struct ColG {
    static constexpr int PT = col_pt(N);
    static constexpr int TPF = N / PT;
    static constexpr int F = kBlock / TPF;
    static constexpr int LDS = F * xlen<N>();  // complex values of exchange space per block
};

// Per-column sum over the TPF threads of each transform, in a fixed order. Within a
// wavefront this is an xor tree. A transform that spans two wavefronts adds the two
// wavefront sums through `red` (2 kBlock/64 doubles of LDS), lower wavefront first.
template <int TPF>
__device__ __forceinline__ void col_sum2(double& a, double& b, double* red) {
    a = wsum_lanes(a, TPF < 64 ? TPF : 64);
    b = wsum_lanes(b, TPF < 64 ? TPF : 64);
    if constexpr (TPF > 64) {
        static_assert(TPF == 128, "transforms span at most two wavefronts");
        const int wave = threadIdx.x / 64;
        if (threadIdx.x % 64 == 0) {
            red[2 * wave] = a;
            red[2 * wave + 1] = b;
        }
        __syncthreads();
        const int w0 = wave & ~1;
        a = red[2 * w0] + red[2 * w0 + 2];
        b = red[2 * w0 + 1] + red[2 * w0 + 3];
        __syncthreads();
    }
}

struct ColPos {
    bool active;
    int l, j, t, f;
};

template <int N>
__device__ __forceinline__ ColPos col_pos(const Shape& sh, int block) {
    using G = ColG<N>;
    ColPos p;
    p.t = threadIdx.x % G::TPF;
    p.f = threadIdx.x / G::TPF;
    const int c = block * G::F + p.f;
    p.active = c < sh.nloops * sh.C;
    p.l = p.active ? c / sh.C : 0;
    p.j = p.active ? c % sh.C : 0;
    return p;
}

// The band values of this thread's slots of column (l, j) (zero outside the band or for an
// inactive column), read through band_get. Column passes issue these loads before their
// transforms, so that their latency overlaps the transform instead of following it.
template <int N>
__device__ __forceinline__ void band_prefetch(const Shape& sh, const ColPos& p, const cd* u, int herm0,
                                              cd* out) {
    using G = ColG<N>;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int kk = band_row(p.t + m * G::TPF, N, sh.Ks);
        out[m] = (p.active && kk >= 0) ? band_get(u, p.j, kk, sh.NB, herm0) : cd{0.0, 0.0};
    }
}

// Inverse s-transform of band column values v (already zero outside the band) into X.
template <int N>
__device__ __forceinline__ void col_inverse_store(const Shape& sh, const ColPos& p, cd* v, cd* X, cd* ex,
                                                  const TwCache<N, ColG<N>::PT>& twc) {
    using G = ColG<N>;
    fft<N, G::PT, true>(v, p.t, ex + p.f * xlen<N>(), twc);
    if (p.active) {
        cd* x = X + ((size_t)p.l * sh.C + p.j) * N;
#pragma unroll
        for (int m = 0; m < G::PT; ++m) x[p.t + m * G::TPF] = v[m];
    }
}

template <int N>
__device__ __forceinline__ void col_pass_A(const Shape& sh, int block, const Work& w, cd* ex,
                                           const cd* __restrict__ tw) {
    using G = ColG<N>;
    const ColPos p = col_pos<N>(sh, block);
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    const cd* u = w.U + ((size_t)p.l * sh.C + p.j) * sh.NB;
    cd v[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int kk = band_row(p.t + m * G::TPF, N, sh.Ks);
        v[m] = (p.active && kk >= 0) ? band_get(u, p.j, kk, sh.NB, w.herm0) : cd{0.0, 0.0};
    }
    col_inverse_store<N>(sh, p, v, w.A, ex, twc);
}

// Reverse mode, first pass: the inverse s-transforms of u_hat (into A, as pass A) and of
// i q r_hat from the saved residual (into C, as pass C would leave it), column by column.
// Without WITH_U, A holds u on the s grid already (saved by the forward) and only the
// residual is transformed.
template <int N, bool WITH_U = true>
__device__ __forceinline__ void col_pass_AC(const Shape& sh, int block, const Work& w, cd* ex,
                                            const cd* __restrict__ tw) {
    using G = ColG<N>;
    const ColPos p = col_pos<N>(sh, block);
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    const size_t col = (size_t)p.l * sh.C + p.j;
    const cd* r = w.R + col * sh.NB;
    const double q = kTwoPi * p.j / sh.L;
    cd v[G::PT], rv[G::PT];
    band_prefetch<N>(sh, p, r, 0, rv);  // with WITH_U, in flight during the first transform
    if constexpr (WITH_U) {
        band_prefetch<N>(sh, p, w.U + col * sh.NB, w.herm0, v);
        col_inverse_store<N>(sh, p, v, w.A, ex, twc);
    }
#pragma unroll
    for (int m = 0; m < G::PT; ++m) v[m] = cd{-q * rv[m].y, q * rv[m].x};  // i q r (zero outside the band)
    col_inverse_store<N>(sh, p, v, w.Cb, ex, twc);
}

template <int N>
__device__ __forceinline__ void col_pass_C(const Shape& sh, int block, const double* __restrict__ T, const Work& w,
                                           int mode, double dtau, int scheme, cd* ex, double* red,
                                           const cd* __restrict__ tw) {
    using G = ColG<N>;
    const ColPos p = col_pos<N>(sh, block);
    const size_t col = (size_t)p.l * sh.C + p.j;
    const cd* Bc = w.BD + col * N;
    cd v[G::PT], ub[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) v[m] = p.active ? Bc[p.t + m * G::TPF] : cd{0.0, 0.0};
    band_prefetch<N>(sh, p, w.U + col * sh.NB, w.herm0, ub);  // in flight during the transform
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    fft<N, G::PT, false>(v, p.t, ex + p.f * xlen<N>(), twc);

    const double Tl = p.active ? T[p.l] : 1.0;
    const double invT = 1.0 / Tl;
    const double q = kTwoPi * p.j / sh.L;
    const double q2 = q * q, q4 = q2 * q2;
    const double lamx = -q4 * q4 + 2.0 * q4 * q2 - q4;
    const double invN = 1.0 / N;
    const double wj = (p.j == 0) ? 1.0 : 2.0;
    double Jp = 0.0, dTp = 0.0;
    cd* g = w.G + col * sh.NB;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = p.t + m * G::TPF;
        const int kk = band_row(e, N, sh.Ks);
        cd x{0.0, 0.0};
        if (p.active && kk >= 0) {
            const int k = (e < N / 2) ? e : e - N;
            const double om = kTwoPi * k;
            const cd wh = cscale(v[m], invN);  // (u u_x)_hat
            const cd uu = ub[m];
            const double a = om * invT;
            // r = -(i om/T) u - (u u_x)_hat + (q^2 - q^4) u
            cd r;
            r.x = a * uu.y - wh.x + (q2 - q4) * uu.x;
            r.y = -a * uu.x - wh.y + (q2 - q4) * uu.y;
            Jp += wj * (r.x * r.x + r.y * r.y);
            dTp += wj * om * (uu.x * r.y - uu.y * r.x);  // Re(u_s conj r), u_s = i om u
            if (mode == MODE_RESIDUAL) {
                g[kk] = r;
            } else if (mode >= MODE_GRAD) {
                // G_lin = (-i om/T - q^2 + q^4) r
                cd gl;
                gl.x = a * r.y + (q4 - q2) * r.x;
                gl.y = -a * r.x + (q4 - q2) * r.y;
                if (mode == MODE_STEP) {
                    const double sig = scheme ? 1.0 / (1.0 - dtau * (lamx - a * a)) : 1.0;
                    const double s = dtau * sig;
                    gl = cd{uu.x + s * gl.x, uu.y + s * gl.y};  // U1
                }
                g[kk] = gl;
            }
            x = cd{-q * r.y, q * r.x};  // i q r
        }
        v[m] = x;
    }
    col_sum2<G::TPF>(Jp, dTp, red);
    if (p.active && p.t == 0) {
        w.partial[2 * col] = Jp;
        w.partial[2 * col + 1] = dTp;
    }
    if (mode >= MODE_GRAD) col_inverse_store<N>(sh, p, v, w.Cb, ex, twc);
}

template <int N>
__device__ __forceinline__ void col_pass_E(const Shape& sh, int block, const Work& w, int mode, double dtau,
                                           int scheme, bool fuseA, cd* ex, const cd* __restrict__ tw,
                                           const double* __restrict__ T = nullptr) {
    using G = ColG<N>;
    const ColPos p = col_pos<N>(sh, block);
    const size_t col = (size_t)p.l * sh.C + p.j;
    const cd* Dc = w.BD + col * N;
    cd v[G::PT], gb[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) v[m] = p.active ? Dc[p.t + m * G::TPF] : cd{0.0, 0.0};
    // G_lin or (reverse mode) the saved residual, in flight during the transform. In the step
    // (U1, then the next step's pass A on the new column) the loads issued after the transform
    // measured faster: pass E at 256 x 1024 took 70.4 us against 75.8 with them in flight.
    if (mode != MODE_STEP) band_prefetch<N>(sh, p, (mode == MODE_ADJOINT ? w.R : w.G) + col * sh.NB, 0, gb);
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    fft<N, G::PT, false>(v, p.t, ex + p.f * xlen<N>(), twc);
    if (mode == MODE_STEP) band_prefetch<N>(sh, p, w.G + col * sh.NB, 0, gb);

    const double invN = 1.0 / N;
    const double q = kTwoPi * p.j / sh.L;
    const double q2 = q * q, q4 = q2 * q2;
    const double lamx = -q4 * q4 + 2.0 * q4 * q2 - q4;
    const double Tl = (mode == MODE_STEP && p.active) ? w.Told[p.l] : (mode == MODE_ADJOINT && p.active) ? T[p.l] : 1.0;
    // reverse mode: G_1 scaled by -gJ_l w_j L, the gradient of sum_l gJ_l J_l in torch's
    // complex convention (gJ folded in by the caller as scale_l = -gJ_l L)
    const double sc = (mode == MODE_ADJOINT && p.active) ? (w.gJ ? -w.gJ[p.l] : -1.0) * sh.L * (p.j == 0 ? 1.0 : 2.0)
                                                         : 1.0;
    cd* g = w.G + col * sh.NB;
    cd* u = w.U + col * sh.NB;
    if (mode == MODE_ADJOINT && w.grad_T && p.active && p.j == 0 && p.t == 0)
        w.grad_T[p.l] = (w.gJ ? w.gJ[p.l] : 1.0) * w.dJdT_in[p.l];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = p.t + m * G::TPF;
        const int kk = band_row(e, N, sh.Ks);
        cd x{0.0, 0.0};
        if (p.active && kk >= 0) {
            const cd ph = cscale(v[m], invN);  // (u r_x)_hat
            if (mode == MODE_ADJOINT) {
                // G_lin = (-i om/T - q^2 + q^4) r, as pass C forms it, then G_1 = G_lin - p_hat
                const cd rr = gb[m];
                const int k = (e < N / 2) ? e : e - N;
                const double a = kTwoPi * k * (1.0 / Tl);
                cd gl;
                gl.x = a * rr.y + (q4 - q2) * rr.x;
                gl.y = -a * rr.x + (q4 - q2) * rr.y;
                const cd g1 = csub(gl, ph);
                g[kk] = cd{sc * g1.x, sc * g1.y};
                v[m] = x;
                continue;
            }
            const cd gg = gb[m];
            if (mode == MODE_STEP) {
                double sig = 1.0;
                if (scheme) {
                    const int k = (e < N / 2) ? e : e - N;
                    const double a = kTwoPi * k / Tl;
                    sig = 1.0 / (1.0 - dtau * (lamx - a * a));
                }
                const double s = dtau * sig;
                x = cd{gg.x - s * ph.x, gg.y - s * ph.y};  // u_hat' = U1 - dtau sigma p_hat
                u[kk] = x;
            } else {
                g[kk] = csub(gg, ph);  // G_1 = G_lin - p_hat
            }
        }
        v[m] = x;
    }
    if (mode == MODE_STEP && fuseA) col_inverse_store<N>(sh, p, v, w.A, ex, twc);
}

// ---------------------------------------------------------------------------- row passes
// TPF = M/PT threads per row transform, P = kBlock / TPF pairs of rows per block, thread
// tid -> t = tid % TPF, p = tid / TPF. A block covers ROWS = 2P consecutive global rows
// g0 .. g0 + 2P - 1 (g = l * N + n, loop-major), paired as (g0 + p, g0 + P + p).
template <int M, int PT_ = (M >= 1024 ? 16 : 8)>
struct RowG {
    static constexpr int PT = PT_;
    static constexpr int TPF = M / PT;  // <= 64: one transform per wavefront at most
    static constexpr int P = kBlock / TPF;
    static constexpr int ROWS = 2 * P;
    static constexpr int CMAX = (M - 1) / 3 + 1;
    static constexpr int TS = ROWS + 1;  // padded row stride of a tile [j][r]
    static constexpr int TILE = CMAX * TS;
    static constexpr int XL = P * xlen<M>();
    // LDS: two input tiles, aliased afterwards by the exchange regions and the output tile
    static constexpr int LDS = (2 * TILE > XL ? 2 * TILE : XL);
    static constexpr int LDS_B = (TILE > XL ? TILE : XL);  // pass B holds one input tile
    static constexpr int PW = 64 / TPF;                   // pairs per wavefront
    static constexpr int NOUT = (2 * PW * CMAX + 63) / 64;  // split outputs per thread
};

// Load rows [g0, g0 + ROWS) of NT intermediates X[0..NT) into tiles tile + i * TILE, laid
// out [j][r] with stride TS, coalesced along n. Rows past nrows read as zero. issue() puts
// every global load of the tile in flight (into registers); commit() stores them to LDS, so
// a caller can do other work while the loads travel. ROWS and N are powers of two, and the
// row passes' column count C = (M-1)/3 + 1 is CMAX. Tiles start at multiples of ROWS, so when
// N >= ROWS a tile lies inside one loop and its elements sit at j N + r from the tile's first
// row (32-bit offsets); shorter loops take the general row-by-row address.
template <int ROWS, int CMAX, int TS, int TILE, int NT>
struct RowTiles {
    static constexpr int NL = (ROWS * CMAX + kBlock - 1) / kBlock;
    static constexpr int n = ROWS * CMAX;
    cd buf[NT][NL];
    __device__ __forceinline__ void issue(const cd* const (&X)[NT], size_t g0, const Shape& sh, size_t nrows) {
        if (sh.N >= ROWS) {
            const size_t base = ((g0 >> sh.logN) * CMAX) * sh.N + (g0 & (size_t)(sh.N - 1));
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int i = threadIdx.x + k * kBlock;
                const int j = i / ROWS, r = i % ROWS;
                const bool ok = (n % kBlock == 0 || i < n) && g0 < nrows;
#pragma unroll
                for (int q = 0; q < NT; ++q) buf[q][k] = ok ? X[q][base + (j * sh.N + r)] : cd{0.0, 0.0};
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int i = threadIdx.x + k * kBlock;
            const int j = i / ROWS, r = i % ROWS;
            const size_t g = g0 + r;
            const bool ok = i < n && g < nrows;
            const size_t off = ok ? ((g >> sh.logN) * CMAX + j) * sh.N + (g & (size_t)(sh.N - 1)) : 0;
#pragma unroll
            for (int q = 0; q < NT; ++q) buf[q][k] = ok ? X[q][off] : cd{0.0, 0.0};
        }
    }
    __device__ __forceinline__ void commit(cd* tile, const Shape&) const {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int i = threadIdx.x + k * kBlock;
            if (n % kBlock == 0 || i < n) {
                const int j = i / ROWS, r = i % ROWS;
#pragma unroll
                for (int q = 0; q < NT; ++q) tile[q * TILE + j * TS + r] = buf[q][k];
            }
        }
    }
};

template <int ROWS, int CMAX, int TS, int TILE, int NT>
__device__ __forceinline__ void load_rows(cd* tile, const cd* const (&X)[NT], size_t g0, const Shape& sh,
                                          size_t nrows) {
    RowTiles<ROWS, CMAX, TS, TILE, NT> ld;
    ld.issue(X, g0, sh, nrows);
    ld.commit(tile, sh);
}

// The same tiles as load_rows, copied by the load unit straight into LDS
// (global_load_lds_dwordx4: lane i of a wavefront writes 16 bytes at the instruction's LDS
// base + 16 i). One wavefront instruction moves 64 consecutive rows of one column j to
// tile[j][r0 .. r0 + 63], so ROWS must be a multiple of 64. Nothing passes through vector
// registers. Lanes whose row lies past nrows store zeros with ordinary LDS writes instead.
// With WAIT the wavefront waits for its own copies before returning (otherwise the caller
// waits for vmcnt(0) itself); the caller's barrier then makes every wavefront's copies
// visible to the block.
template <int ROWS, int CMAX, int TS, int TILE, int NT, bool WAIT = true>
__device__ __forceinline__ void load_rows_lds(cd* tile, const cd* const (&X)[NT], size_t g0, const Shape& sh,
                                              size_t nrows) {
    static_assert(ROWS % 64 == 0, "a copy instruction covers 64 rows of one column");
    constexpr int RC = ROWS / 64;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    constexpr int per_field = CMAX * RC;
    const size_t g = g0 + lane;
    for (int k = wave; k < NT * per_field; k += kBlock / 64) {
        const int q = k / per_field, rem = k % per_field;
        const int j = rem / RC, r0 = (rem % RC) * 64;
        cd* dst = tile + q * TILE + j * TS + r0;
        const size_t gr = g + r0;
        if (gr < nrows) {
            const cd* src = X[q] + ((gr >> sh.logN) * CMAX + j) * sh.N + (gr & (size_t)(sh.N - 1));
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)const_cast<cd*>(src),
                                             (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        } else {
            dst[lane] = cd{0.0, 0.0};
        }
    }
    if constexpr (WAIT) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Store tile[j][r] (stride TS) to rows [g0, g0 + ROWS) of X, addressed as RowTiles loads them.
template <int ROWS, int CMAX>
__device__ __forceinline__ void store_rows(const cd* tile, int TS, cd* X, size_t g0, const Shape& sh,
                                           size_t nrows) {
    constexpr int NL = (ROWS * CMAX + kBlock - 1) / kBlock;
    constexpr int n = ROWS * CMAX;
    if (sh.N >= ROWS) {
        if (g0 >= nrows) return;
        cd* base = X + ((g0 >> sh.logN) * CMAX) * sh.N + (g0 & (size_t)(sh.N - 1));
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int i = threadIdx.x + k * kBlock;
            const int j = i / ROWS, r = i % ROWS;
            if (n % kBlock == 0 || i < n) base[j * sh.N + r] = tile[j * TS + r];
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * kBlock;
        const int j = i / ROWS, r = i % ROWS;
        const size_t g = g0 + r;
        if (i < n && g < nrows)
            X[((g >> sh.logN) * CMAX + j) * sh.N + (g & (size_t)(sh.N - 1))] = tile[j * TS + r];
    }
}

// Element e of the Hermitian extension of half spectrum tile[j][r] (j < C; X_0 read as real):
// tile[e] for e <= Kx, conj(tile[M - e]) for e >= M - Kx, zero between. Written without
// branches (one read of a valid element, then selects), since e differs across the lanes of
// a transform.
__device__ __forceinline__ cd herm_ext(const cd* tile, int TS, int r, int e, int M, int Kx) {
    const int j = e <= M / 2 ? e : M - e;  // |frequency|
    const bool in = j <= Kx;
    const cd v = tile[(in ? j : 0) * TS + r];
    const double y = e == 0 ? 0.0 : (e > M / 2 ? -v.y : v.y);
    return in ? cd{v.x, y} : cd{0.0, 0.0};
}

// Spectrum of f + i g for two real rows f, g given by their half spectra (packed complex).
__device__ __forceinline__ cd pack2(cd f, cd g) { return cd{f.x - g.y, f.y + g.x}; }

// herm_ext for the elements e = t + m TPF (m = 0 .. PT-1) that thread t of a row transform
// holds, with the band limit Kx = (M-1)/3 of an M-point row known at compile time. A slot
// whose elements all lie in the band reads them directly (e <= Kx) or as conjugates of their
// partners (e >= M - Kx); a slot wholly outside the band is zero; only a slot that straddles
// a band edge selects per lane. The values are herm_ext's, bit for bit.
template <int M, int PT, int m>
__device__ __forceinline__ cd herm_slot(const cd* tile, int TS, int r, int t) {
    constexpr int TPF = M / PT, Kx = (M - 1) / 3;
    constexpr int lo = m * TPF, hi = lo + TPF - 1;
    if constexpr (hi <= Kx) {
        const cd v = tile[(lo + t) * TS + r];
        if constexpr (lo == 0) return cd{v.x, t == 0 ? 0.0 : v.y};  // X_0 is read as real
        return v;
    } else if constexpr (lo >= M - Kx) {
        const cd v = tile[(M - lo - t) * TS + r];
        return cd{v.x, -v.y};
    } else if constexpr (lo > Kx && hi < M - Kx) {
        return cd{0.0, 0.0};
    } else {
        return herm_ext(tile, TS, r, lo + t, M, Kx);
    }
}

// va[m] = pack2 of rows ra and rb of a tile, slot by slot (see herm_slot).
template <int M, int PT, int m = 0>
__device__ __forceinline__ void herm_pack(const cd* tile, int TS, int ra, int rb, int t, cd* va) {
    if constexpr (m < PT) {
        va[m] = pack2(herm_slot<M, PT, m>(tile, TS, ra, t), herm_slot<M, PT, m>(tile, TS, rb, t));
        herm_pack<M, PT, m + 1>(tile, TS, ra, rb, t, va);
    }
}

// herm_pack, and in vb the x-derivatives of the same rows (i q times each element, q of the
// signed frequency of slot m).
template <int M, int PT, int m = 0>
__device__ __forceinline__ void herm_pack_dx(const cd* tile, int TS, int ra, int rb, int t, double dq, cd* va,
                                             cd* vb) {
    if constexpr (m < PT) {
        constexpr int TPF = M / PT;
        const int e = t + m * TPF;
        const double q = dq * (double)((e <= M / 2) ? e : e - M);
        const cd a = herm_slot<M, PT, m>(tile, TS, ra, t), b = herm_slot<M, PT, m>(tile, TS, rb, t);
        va[m] = pack2(a, b);
        vb[m] = pack2(cd{-q * a.y, q * a.x}, cd{-q * b.y, q * b.x});
        herm_pack_dx<M, PT, m + 1>(tile, TS, ra, rb, t, dq, va, vb);
    }
}

// Pass B forms u u_x as (1/2) (u^2)_x (two transforms per pair of rows) for rows of up to
// kSquareMaxM points, and as the product u * u_x (three transforms) for longer rows.
// Differentiating the square multiplies the round-off of mode j by q_j / 2, against the
// product's round-off of order |u u_x|: the ratio grows as Kx over the input's dominant mode
// index. Measured against the FP64 oracle on low-mode loops (|j| <= 8), the flow G of the
// square form errs by 1.1e-13 at 128 x 64, 4.9e-13 at 256 x 1024 and 3.8e-12 at 512 x 32
// (normwise), the product form by 1.7e-14, 3.0e-14 and 1.3e-13; with Kx <= 42 the square form
// stays inside the 1e-12 bound even for a loop made of its lowest mode.
constexpr int kSquareMaxM = 128;

// Forward transform of the pair's product values va, then the split of the result
// Z = W_a + i W_b into the two rows' half spectra, W_a(j) = (Z_j + conj Z_{M-j}) / 2 and
// W_b(j) = (Z_j - conj Z_{M-j}) / (2i), scaled by 1/M, written to tile[j][r] over the
// inputs' LDS. With DX the rows' spectra are differentiated on the way, i q_j / 2 W (the half
// derivative of a square).
template <int M, int PT, bool DX>
__device__ __forceinline__ void row_forward_split(const Shape& sh, cd* va, cd* lds, cd* ex, int t,
                                                  const TwCache<M, PT>& twc) {
    using G = RowG<M, PT>;
    fft<M, G::PT, false>(va, t, ex, twc);
#pragma unroll
    for (int m = 0; m < G::PT; ++m) ex[xpos(t + m * G::TPF)] = va[m];
    wave_lds_order();
    const int lane = threadIdx.x % 64;
    const int pw0 = (threadIdx.x / 64) * G::PW;
    constexpr int nout = 2 * G::PW * G::CMAX;
    const double s = 0.5 / M;
    const double hq = (kTwoPi / sh.L) * (0.25 / M);  // q_j / 2 per unit j, with the 1/(2M) of the split
    cd outv[G::NOUT];
#pragma unroll
    for (int i = 0; i < G::NOUT; ++i) {
        const int idx = lane + 64 * i;
        if (idx < nout) {
            const int pp = pw0 + idx / (2 * G::CMAX);
            const int rem = idx % (2 * G::CMAX);
            const int j = rem % G::CMAX;
            const bool rb = rem >= G::CMAX;  // row b (else row a) of the pair
            const cd* e2 = lds + pp * xlen<M>();
            const cd a = e2[xpos(j)];
            const cd b = e2[xpos((M - j) & (M - 1))];
            if constexpr (DX) {
                const double c = hq * j;
                outv[i] = rb ? cd{c * (a.x - b.x), c * (a.y + b.y)} : cd{c * (b.y - a.y), c * (a.x + b.x)};
            } else {
                outv[i] = rb ? cd{(a.y + b.y) * s, (b.x - a.x) * s} : cd{(a.x + b.x) * s, (a.y - b.y) * s};
            }
        }
    }
    __syncthreads();  // every wave is done with its exchange region: reuse as the output tile
#pragma unroll
    for (int i = 0; i < G::NOUT; ++i) {
        const int idx = lane + 64 * i;
        if (idx < nout) {
            const int pp = pw0 + idx / (2 * G::CMAX);
            const int rem = idx % (2 * G::CMAX);
            // consecutive lanes write consecutive j of one row: stride TS, no bank conflicts
            lds[(rem % G::CMAX) * G::TS + (rem >= G::CMAX ? G::P + pp : pp)] = outv[i];
        }
    }
    __syncthreads();
}

// u u_x = (1/2) (u^2)_x on rows a and b of a pair: one inverse transform of u_a + i u_b, the
// squares (u_a^2) + i (u_b^2) in physical space, one forward transform, and the split with the
// factor i q_j / 2. Both fields are band-limited, so (u^2)_x of the band equals the band of
// 2 u u_x exactly; one transform of three is saved.
template <int M, int PT = RowG<M>::PT>
__device__ __forceinline__ void row_square_dx(const Shape& sh, cd* va, cd* lds, int t, int p,
                                              const TwCache<M, PT>& twc) {
    cd* ex = lds + p * xlen<M>();
    __syncthreads();  // every wave has read its inputs from the tile: the tile is free
    fft<M, PT, true>(va, t, ex, twc);
#pragma unroll
    for (int m = 0; m < PT; ++m) va[m] = cd{va[m].x * va[m].x, va[m].y * va[m].y};
    row_forward_split<M, PT, true>(sh, va, lds, ex, t, twc);
}

// Products of two real fields f, g on rows a and b of a pair. The two inverse x-transforms
// take the rows of one field at a time (va = f_a + i f_b, vb = g_a + i g_b), so each transform
// carries values of one scale; packing f and g of one row together would let the round-off
// of the larger (r_x can exceed u by q_max^5) swamp the smaller. Then one forward transform
// of (f_a g_a) + i (f_b g_b) and the split into the two rows' half spectra (scaled by 1/M),
// written to tile[j][r] over the inputs' LDS.
template <int M, int PT = RowG<M>::PT>
__device__ __forceinline__ void row_products(const Shape& sh, cd* va, cd* vb, cd* lds, int t, int p,
                                             const TwCache<M, PT>& twc) {
    using G = RowG<M, PT>;
    cd* ex = lds + p * xlen<M>();
    __syncthreads();  // every wave has read its inputs from the tiles: the tiles are free
    fft<M, G::PT, true>(va, t, ex, twc);
    fft<M, G::PT, true>(vb, t, ex, twc);
#pragma unroll
    for (int m = 0; m < G::PT; ++m) va[m] = cd{va[m].x * vb[m].x, va[m].y * vb[m].y};
    row_forward_split<M, PT, false>(sh, va, lds, ex, t, twc);
}

// DMA selects load_rows_lds over load_rows (tiles of 64 rows or more). PT below the default
// spreads each row transform over more threads: tiles are then shorter, and a block covers
// the rows of one default-size tile (so that tile indices keep their meaning) in SUB
// consecutive sub-tiles.
template <int M, bool DMA = false, int PT = RowG<M>::PT>
__device__ __forceinline__ void row_pass_B(const Shape& sh, int block, const Work& w, cd* lds,
                                           const cd* __restrict__ tw) {
    using G = RowG<M, PT>;
    constexpr int SUB = RowG<M>::ROWS / G::ROWS;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const int t = threadIdx.x % G::TPF, p = threadIdx.x / G::TPF;
    TwCache<M, PT> twc;
    tw_cache_load<M, PT>(twc, t, tw);
    auto sub = [&](size_t g0) {
        {
            const cd* const src[1] = {w.A};
            if constexpr (DMA)
                load_rows_lds<G::ROWS, G::CMAX, G::TS, G::TILE, 1>(lds, src, g0, sh, nrows);
            else
                load_rows<G::ROWS, G::CMAX, G::TS, G::TILE, 1>(lds, src, g0, sh, nrows);
        }
        __syncthreads();
        if constexpr (M <= kSquareMaxM) {
            cd va[PT];
            herm_pack<M, PT>(lds, G::TS, p, G::P + p, t, va);  // u, rows a and b
            row_square_dx<M, PT>(sh, va, lds, t, p, twc);
        } else {
            cd va[PT], vb[PT];
            herm_pack_dx<M, PT>(lds, G::TS, p, G::P + p, t, kTwoPi / sh.L, va, vb);  // u and u_x, rows a and b
            row_products<M, PT>(sh, va, vb, lds, t, p, twc);
        }
        store_rows<G::ROWS, G::CMAX>(lds, G::TS, w.BD, g0, sh, nrows);
    };
    const size_t gb = (size_t)block * RowG<M>::ROWS;
    if constexpr (SUB == 1) {
        sub(gb);
    } else {
#pragma unroll 1
        for (int h = 0; h < SUB; ++h) {
            if (h > 0) __syncthreads();  // the previous sub-tile's output tile has been stored
            sub(gb + (size_t)h * G::ROWS);
        }
    }
}

// Sum the per-column partials of loop l into J, dJ/dT; in MODE_STEP also advance T.
// Called by all 64 lanes of one wavefront: lanes add strided partials in a fixed order, then
// an xor tree combines them.
__device__ __forceinline__ void finalize_loop(const Shape& sh, int l, const Work& w, double* T, int mode,
                                              double dtau, double* J_hist, double* Jout, double* dJdTout) {
    const int lane = threadIdx.x % 64;
    const double* pp = w.partial + (size_t)l * sh.C * 2;
    double sj = 0.0, st = 0.0;
    for (int j = lane; j < sh.C; j += 64) {
        sj += pp[2 * j];
        st += pp[2 * j + 1];
    }
    sj = wsum_lanes(sj, 64);
    st = wsum_lanes(st, 64);
    if (lane != 0) return;
    const double Tl = T[l];
    const double J = 0.5 * sh.L * sj;
    const double dJdT = sh.L * st / (Tl * Tl);
    w.J[l] = J;
    w.dJdT[l] = dJdT;
    if (Jout) Jout[l] = J;
    if (dJdTout) dJdTout[l] = dJdT;
    bool bad = !(Tl > 0.0) || !isfinite(Tl) || !isfinite(J) || !isfinite(dJdT);
    if (mode == MODE_STEP) {
        const double Tn = Tl - dtau * dJdT;
        w.Told[l] = Tl;
        T[l] = Tn;
        if (J_hist) J_hist[l] = J;
        bad = bad || !(Tn > 0.0) || !isfinite(Tn);
    }
    if (bad) atomicCAS(w.status, 0, -4);
}

template <int M, bool DMA = false, int PT = RowG<M>::PT>
__device__ __forceinline__ void row_pass_D(const Shape& sh, int block, const Work& w, double* T, int mode,
                                           double dtau, double* J_hist, double* Jout, double* dJdTout, cd* lds,
                                           const cd* __restrict__ tw) {
    using G = RowG<M, PT>;
    constexpr int SUB = RowG<M>::ROWS / G::ROWS;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const size_t gb = (size_t)block * RowG<M>::ROWS;
    // Loops whose first row lies in this block are finished here (partials from pass C), by
    // wavefront 0 while the first sub-tile's loads are in flight.
    auto finalize = [&]() {
        if (mode != MODE_ADJOINT && threadIdx.x < 64) {
            const size_t l0 = (gb + sh.N - 1) >> sh.logN;  // first loop starting at or after gb
            for (size_t l = l0; (l << sh.logN) < gb + RowG<M>::ROWS && l < (size_t)sh.nloops; ++l)
                finalize_loop(sh, (int)l, w, T, mode, dtau, J_hist, Jout, dJdTout);
        }
    };
    cd* tA = lds;
    cd* tC = lds + G::TILE;
    const int t = threadIdx.x % G::TPF, p = threadIdx.x / G::TPF;
    TwCache<M, PT> twc;
    tw_cache_load<M, PT>(twc, t, tw);
    auto sub = [&](size_t g0, bool first) {
        {
            const cd* const src[2] = {w.A, w.Cb};
            if constexpr (DMA) {
                load_rows_lds<G::ROWS, G::CMAX, G::TS, G::TILE, 2, false>(tA, src, g0, sh, nrows);
                if (first) finalize();
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            } else {
                RowTiles<G::ROWS, G::CMAX, G::TS, G::TILE, 2> ld;
                ld.issue(src, g0, sh, nrows);
                if (first) finalize();
                ld.commit(tA, sh);
            }
        }
        __syncthreads();
        cd va[PT], vb[PT];
        herm_pack<M, PT>(tA, G::TS, p, G::P + p, t, va);  // u
        herm_pack<M, PT>(tC, G::TS, p, G::P + p, t, vb);  // r_x
        row_products<M, PT>(sh, va, vb, lds, t, p, twc);
        store_rows<G::ROWS, G::CMAX>(lds, G::TS, w.BD, g0, sh, nrows);
    };
    if constexpr (SUB == 1) {
        sub(gb, true);
    } else {
#pragma unroll 1
        for (int h = 0; h < SUB; ++h) {
            if (h > 0) __syncthreads();  // the previous sub-tile's output tile has been stored
            sub(gb + (size_t)h * G::ROWS, h == 0);
        }
    }
}

}  // namespace lo
