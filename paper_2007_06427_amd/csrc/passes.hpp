// The five passes of one fictitious-time step of the KS loop dynamics, as block-level device
// functions over one tile of a uniform batch of loops (Sec. 4.2 of Azimi, Ashtari &
// Schneider, arXiv:2007.06427).
//
// Notation: M = Nx and N = Ns grid points. The band is |j| <= Kx and |k| <= Ks, with
// Kx = (M-1)/3 and Ks = (N-1)/3. C = Kx + 1 is the number of retained non-negative spatial
// modes. q_j = 2 pi j / L and omega_k = 2 pi k.
//
// Pass A (columns): A(j, s_n) = sum_k u_hat_{j,k} e^{2 pi i n k / N}, an inverse s-transform
//                   of each retained column j.
// Pass B (rows):    u and u_x at (x_m, s_n) from inverse x-transforms of A(., s_n) and of
//                   i q A(., s_n); then w = u u_x; B(j, s_n) = forward x-transform of w, kept
//                   for j < C.
// Pass C (columns): w_hat = forward s-transform of B. Then the residual of eq. KS_R,
//                     r_hat = -(i omega/T) u_hat - w_hat + q^2 u_hat - q^4 u_hat.
//                   Forming u u_x itself rather than (1/2) d/dx (u^2) keeps the round-off of
//                   the high modes at the size of the product, not amplified by q_max.
//                   Per-column partial sums of J and dJ/dT. The linear part of the flow,
//                     G_lin = (-i omega/T - q^2 + q^4) r_hat.
//                   C(j, s_n) = inverse s-transform of i q r_hat, which is r_x by columns.
// Pass D (rows):    u and r_x at each row, p = u r_x, D(j, s_n) = forward x-transform of p.
//                   The first block of each loop also finishes J and dJ/dT.
// Pass E (columns): p_hat = forward s-transform of D, so G_1 = G_lin - p_hat (eq. KS_G).
//                   Optionally the Euler / semi-implicit Euler update (Sec. 4.2).
//
// Every product is of two band-limited fields on the full grid, so it is free of aliasing
// in the band. Truncation to the band is implicit: only retained modes are ever formed.
//
// Layouts (complex, interleaved doubles):
//   state   uhat[l][k mod N][j],  j = 0 .. M/2     (rfft layout, the C-ABI format)
//   A,B,C,D X[l][n][j],           j = 0 .. C-1     (row-major, j fastest)
//   G_lin   G[l][kk][j],          kk = k for k >= 0, kk = k + 2 Ks + 1 for k < 0
#pragma once

#include "fft.hpp"

namespace lo {

constexpr int kBlock = 256;  // threads per block for every pass kernel

enum Mode : int {
    MODE_RESIDUAL = 0,  // pass C writes r_hat to the output array
    MODE_COST = 1,      // pass C partials only
    MODE_GRAD = 2,      // pass E writes G_1
    MODE_STEP = 3,      // pass D updates T, pass E updates u_hat
};

struct Shape {
    int M, N;      // grid points in x and s
    int Kx, Ks;    // band limits
    int H;         // M/2 + 1 columns of the rfft layout
    int C;         // Kx + 1 retained columns
    int nloops;
    double L;
};

struct Work {
    cd* A;           // [nloops][N][C]
    cd* BD;          // [nloops][N][C]   (B, then D)
    cd* Cb;          // [nloops][N][C]
    cd* Glin;        // [nloops][2Ks+1][C]
    double* partial; // [nloops][C][2]   per-column sums: w_j |r|^2 and w_j Re(u_s conj r)
    double* J;       // [nloops]
    double* dJdT;    // [nloops]
    double* Told;    // [nloops]   period at the start of the current step
    int* status;     // sticky device status
};

constexpr double kTwoPi = 6.283185307179586476925286766559005768;

// ---------------------------------------------------------------------------- state access
// u_hat_{j,k} for in-band (j, k) at FFT-order row e, column 0 read through its Hermitian part.
__device__ __forceinline__ cd load_state(const cd* __restrict__ u, int e, int j, int N, int H) {
    cd v = u[(size_t)e * H + j];
    if (j == 0) {
        cd p = u[(size_t)((N - e) & (N - 1)) * H];
        v = cd{0.5 * (v.x + p.x), 0.5 * (v.y - p.y)};
    }
    return v;
}

__device__ __forceinline__ int band_row(int e, int N, int Ks) {
    // compact row index kk of FFT-order row e, or -1 outside the band
    if (e <= Ks) return e;
    if (e >= N - Ks) return e - (N - 2 * Ks - 1);
    return -1;
}

// ---------------------------------------------------------------------------- column passes
// Block layout for columns: F = 2048 / N transforms of length N, N/8 threads each.
// Thread tid -> slot f = tid % F (column within the block), t = tid / F.
// Global column index c = blockIdx * F + f runs over nloops * C columns (loop-major).
template <int N>
struct ColGeom {
    static constexpr int TPF = N / 8;
    static constexpr int F = kBlock / TPF;
};

template <int N>
__device__ __forceinline__ void col_pass_A(const Shape& sh, int block, const cd* __restrict__ uhat,
                                           const Work& w, cd* ex, const cd* __restrict__ tw) {
    using G = ColGeom<N>;
    const int f = threadIdx.x % G::F, t = threadIdx.x / G::F;
    const int c = block * G::F + f;
    const bool active = c < sh.nloops * sh.C;
    const int l = active ? c / sh.C : 0, j = active ? c % sh.C : 0;
    const cd* u = uhat + (size_t)l * N * sh.H;
    cd v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int e = t + m * G::TPF;
        v[m] = (active && band_row(e, N, sh.Ks) >= 0) ? load_state(u, e, j, N, sh.H) : cd{0.0, 0.0};
    }
    fft<N, true>(v, t, ex + f, G::F, tw);
    if (active) {
        cd* A = w.A + (size_t)l * N * sh.C;
#pragma unroll
        for (int m = 0; m < 8; ++m) A[(size_t)(t + m * G::TPF) * sh.C + j] = v[m];
    }
}

// Deterministic per-column sum over the N/8 threads of each transform (fixed tree order).
template <int N>
__device__ __forceinline__ void col_reduce2(double a, double b, double* red, double* out, bool active, int c) {
    using G = ColGeom<N>;
    const int f = threadIdx.x % G::F, t = threadIdx.x / G::F;
    __syncthreads();  // red aliases the exchange buffer
    red[t * G::F + f] = a;
    red[kBlock + t * G::F + f] = b;
    __syncthreads();
#pragma unroll
    for (int s = G::TPF / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[t * G::F + f] += red[(t + s) * G::F + f];
            red[kBlock + t * G::F + f] += red[kBlock + (t + s) * G::F + f];
        }
        __syncthreads();
    }
    if (t == 0 && active) {
        out[2 * c] = red[f];
        out[2 * c + 1] = red[kBlock + f];
    }
    __syncthreads();
}

template <int N>
__device__ __forceinline__ void col_pass_C(const Shape& sh, int block, const cd* __restrict__ uhat,
                                           const double* __restrict__ T, const Work& w, cd* rhat_out,
                                           int mode, cd* ex, const cd* __restrict__ tw) {
    using G = ColGeom<N>;
    const int f = threadIdx.x % G::F, t = threadIdx.x / G::F;
    const int c = block * G::F + f;
    const bool active = c < sh.nloops * sh.C;
    const int l = active ? c / sh.C : 0, j = active ? c % sh.C : 0;
    const cd* u = uhat + (size_t)l * N * sh.H;
    const cd* B = w.BD + (size_t)l * N * sh.C;
    cd v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m)
        v[m] = active ? B[(size_t)(t + m * G::TPF) * sh.C + j] : cd{0.0, 0.0};
    fft<N, false>(v, t, ex + f, G::F, tw);

    const double Tl = active ? T[l] : 1.0;
    const double invT = 1.0 / Tl;
    const double q = kTwoPi * j / sh.L;
    const double q2 = q * q, q4 = q2 * q2;
    const double invN = 1.0 / N;
    const double wj = (j == 0) ? 1.0 : 2.0;
    double Jp = 0.0, dTp = 0.0;
    cd* Gl = w.Glin + (size_t)l * (2 * sh.Ks + 1) * sh.C;
    cd* R = rhat_out ? rhat_out + (size_t)l * N * sh.H : nullptr;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int e = t + m * G::TPF;
        const int kk = band_row(e, N, sh.Ks);
        cd x{0.0, 0.0};
        if (active && kk >= 0) {
            const int k = (e < N / 2) ? e : e - N;
            const double om = kTwoPi * k;
            const cd wh = cscale(v[m], invN);
            const cd uu = load_state(u, e, j, N, sh.H);
            const double a = om * invT;
            // r = -(i om/T) u - (u u_x)_hat + (q^2 - q^4) u
            cd r;
            r.x = a * uu.y - wh.x + (q2 - q4) * uu.x;
            r.y = -a * uu.x - wh.y + (q2 - q4) * uu.y;
            Jp += wj * (r.x * r.x + r.y * r.y);
            // u_s = i om u ;  Re(u_s conj r)
            dTp += wj * om * (-uu.y * r.x + uu.x * r.y);
            // G_lin = (-i om/T - q^2 + q^4) r
            if (mode >= MODE_GRAD) {
                cd g;
                g.x = a * r.y + (q4 - q2) * r.x;
                g.y = -a * r.x + (q4 - q2) * r.y;
                Gl[(size_t)kk * sh.C + j] = g;
            }
            if (R) R[(size_t)e * sh.H + j] = r;
            x = cd{-q * r.y, q * r.x};  // i q r
        } else if (active && R) {
            R[(size_t)e * sh.H + j] = cd{0.0, 0.0};
        }
        v[m] = x;
    }
    col_reduce2<N>(Jp, dTp, reinterpret_cast<double*>(ex), w.partial, active, c);
    if (mode >= MODE_GRAD) {
        fft<N, true>(v, t, ex + f, G::F, tw);
        if (active) {
            cd* Cb = w.Cb + (size_t)l * N * sh.C;
#pragma unroll
            for (int m = 0; m < 8; ++m) Cb[(size_t)(t + m * G::TPF) * sh.C + j] = v[m];
        }
    }
}

template <int N>
__device__ __forceinline__ void col_pass_E(const Shape& sh, int block, cd* uhat, const Work& w, cd* Gout,
                                           int mode, double dtau, int scheme, cd* ex,
                                           const cd* __restrict__ tw) {
    using G = ColGeom<N>;
    const int f = threadIdx.x % G::F, t = threadIdx.x / G::F;
    const int c = block * G::F + f;
    const bool active = c < sh.nloops * sh.C;
    const int l = active ? c / sh.C : 0, j = active ? c % sh.C : 0;
    const cd* D = w.BD + (size_t)l * N * sh.C;
    cd v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m)
        v[m] = active ? D[(size_t)(t + m * G::TPF) * sh.C + j] : cd{0.0, 0.0};
    fft<N, false>(v, t, ex + f, G::F, tw);
    if (!active) return;

    const cd* Gl = w.Glin + (size_t)l * (2 * sh.Ks + 1) * sh.C;
    const double invN = 1.0 / N;
    const double q = kTwoPi * j / sh.L;
    const double q2 = q * q, q4 = q2 * q2;
    const double lamx = -q4 * q4 + 2.0 * q4 * q2 - q4;
    const double Tl = (mode == MODE_STEP) ? w.Told[l] : 1.0;
    cd* u = uhat + (size_t)l * N * sh.H;
    cd* Go = Gout ? Gout + (size_t)l * N * sh.H : nullptr;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int e = t + m * G::TPF;
        const int kk = band_row(e, N, sh.Ks);
        if (kk >= 0) {
            const cd p = cscale(v[m], invN);
            const cd gl = Gl[(size_t)kk * sh.C + j];
            const cd g = csub(gl, p);
            if (Go) Go[(size_t)e * sh.H + j] = g;
            if (mode == MODE_STEP) {
                double sig = 1.0;
                if (scheme == 1) {
                    const int k = (e < N / 2) ? e : e - N;
                    const double a = kTwoPi * k / Tl;
                    const double lam = -a * a + lamx;
                    sig = 1.0 / (1.0 - dtau * lam);
                }
                const double s = dtau * sig;
                cd uu = u[(size_t)e * sh.H + j];
                uu.x += s * g.x;
                uu.y += s * g.y;
                u[(size_t)e * sh.H + j] = uu;
            }
        } else if (Go) {
            Go[(size_t)e * sh.H + j] = cd{0.0, 0.0};
        }
    }
}

// ---------------------------------------------------------------------------- row passes
// Block layout for rows: P = 2048 / M pairs of rows, M/8 threads per pair-transform.
// Thread tid -> pair p = tid % P, t = tid / P. A block covers 2P consecutive global rows
// g0 .. g0 + 2P - 1 (g = l * N + n, loop-major), paired as (g0 + p, g0 + P + p).
template <int M>
struct RowGeom {
    static constexpr int TPF = M / 8;
    static constexpr int P = kBlock / TPF;
    static constexpr int ROWS = 2 * P;
    static constexpr int CMAX = (M - 1) / 3 + 1;
};

// Element e of the Hermitian extension of a half spectrum X[0..C-1] (X[0] read as real).
__device__ __forceinline__ cd herm_ext(const cd* X, int e, int M, int Kx) {
    if (e == 0) return cd{X[0].x, 0.0};
    if (e <= Kx) return X[e];
    if (e >= M - Kx) return cconj(X[M - e]);
    return cd{0.0, 0.0};
}

// Load a tile of rows [g0, g0 + rows) of an intermediate into LDS, coalesced.
__device__ __forceinline__ void load_tile(cd* tile, const cd* __restrict__ X, size_t g0, int rows, int C,
                                          size_t nrows) {
    const size_t base = g0 * C;
    const int n = rows * C;
    const size_t lim = nrows * C;
    for (int i = threadIdx.x; i < n; i += kBlock) tile[i] = (base + i < lim) ? X[base + i] : cd{0.0, 0.0};
}

// Forward transform of packed real pair z = w_a + i w_b held in v, written as the two half
// spectra W_a, W_b (scaled by 1/M) to rows ga, gb of Y. ex must be free.
template <int M>
__device__ __forceinline__ void row_forward_store(cd v[8], int t, int p, cd* ex, const cd* __restrict__ tw,
                                                  cd* Y, size_t g0, size_t nrows, int C) {
    using G = RowGeom<M>;
    fft<M, false>(v, t, ex + p, G::P, tw);
#pragma unroll
    for (int m = 0; m < 8; ++m) ex[(t + m * G::TPF) * G::P + p] = v[m];
    __syncthreads();
    const double s = 0.5 / M;
    for (int i = threadIdx.x; i < G::P * C; i += kBlock) {
        const int pp = i / C, j = i % C;
        const cd a = ex[j * G::P + pp];
        const cd b = ex[((M - j) & (M - 1)) * G::P + pp];
        // W_a = (Z_j + conj(Z_{M-j})) / 2,  W_b = (Z_j - conj(Z_{M-j})) / (2i)
        const cd wa{(a.x + b.x) * s, (a.y - b.y) * s};
        const cd wb{(a.y + b.y) * s, (b.x - a.x) * s};
        const size_t ga = g0 + pp, gb = g0 + G::P + pp;
        if (ga < nrows) Y[ga * C + j] = wa;
        if (gb < nrows) Y[gb * C + j] = wb;
    }
}

// Element e of i q_j times the Hermitian extension of X (the x-derivative's spectrum).
__device__ __forceinline__ cd herm_ext_dx(const cd* X, int e, int M, int Kx, double dq) {
    const cd v = herm_ext(X, e, M, Kx);
    const double q = dq * (double)((e <= M / 2) ? e : e - M);
    return cd{-q * v.y, q * v.x};
}

template <int M>
__device__ __forceinline__ void row_pass_B(const Shape& sh, int block, const Work& w, cd* tile, cd* ex,
                                           const cd* __restrict__ tw) {
    using G = RowGeom<M>;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const size_t g0 = (size_t)block * G::ROWS;
    load_tile(tile, w.A, g0, G::ROWS, sh.C, nrows);
    __syncthreads();
    const int p = threadIdx.x % G::P, t = threadIdx.x / G::P;
    const double dq = kTwoPi / sh.L;
    cd va[8], vb[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int e = t + m * G::TPF;
        const cd* Xa = tile + p * sh.C;
        const cd* Xb = tile + (G::P + p) * sh.C;
        cd a = herm_ext(Xa, e, M, sh.Kx), b = herm_ext_dx(Xa, e, M, sh.Kx, dq);
        va[m] = cd{a.x - b.y, a.y + b.x};  // u_hat + i (u_x)_hat, row a
        a = herm_ext(Xb, e, M, sh.Kx);
        b = herm_ext_dx(Xb, e, M, sh.Kx, dq);
        vb[m] = cd{a.x - b.y, a.y + b.x};  // row b
    }
    fft<M, true>(va, t, ex + p, G::P, tw);
    fft<M, true>(vb, t, ex + p, G::P, tw);
#pragma unroll
    for (int m = 0; m < 8; ++m) va[m] = cd{va[m].x * va[m].y, vb[m].x * vb[m].y};  // (u u_x)_a + i (u u_x)_b
    row_forward_store<M>(va, t, p, ex, tw, w.BD, g0, nrows, sh.C);
}

// Sum the per-column partials of loop l into J, dJ/dT; in MODE_STEP also advance T.
__device__ __forceinline__ void finalize_loop(const Shape& sh, int l, const Work& w, double* T, int mode,
                                              double dtau, double* J_hist, double* Jout, double* dJdTout) {
    const double* pp = w.partial + (size_t)l * sh.C * 2;
    double sj = 0.0, st = 0.0;
    for (int j = 0; j < sh.C; ++j) {
        sj += pp[2 * j];
        st += pp[2 * j + 1];
    }
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

template <int M>
__device__ __forceinline__ void row_pass_D(const Shape& sh, int block, const Work& w, double* T, int mode,
                                           double dtau, double* J_hist, double* Jout, double* dJdTout,
                                           cd* tile, cd* ex, const cd* __restrict__ tw) {
    using G = RowGeom<M>;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const size_t g0 = (size_t)block * G::ROWS;
    // loops whose first row lies in this block are finished here (partials from pass C)
    for (int i = threadIdx.x; i < G::ROWS; i += kBlock) {
        const size_t g = g0 + i;
        if (g < nrows && (g % sh.N) == 0)
            finalize_loop(sh, (int)(g / sh.N), w, T, mode, dtau, J_hist, Jout, dJdTout);
    }
    cd* tileA = tile;
    cd* tileC = tile + G::ROWS * G::CMAX;
    load_tile(tileA, w.A, g0, G::ROWS, sh.C, nrows);
    load_tile(tileC, w.Cb, g0, G::ROWS, sh.C, nrows);
    __syncthreads();
    const int p = threadIdx.x % G::P, t = threadIdx.x / G::P;
    cd va[8], vb[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int e = t + m * G::TPF;
        cd a = herm_ext(tileA + p * sh.C, e, M, sh.Kx), b = herm_ext(tileC + p * sh.C, e, M, sh.Kx);
        va[m] = cd{a.x - b.y, a.y + b.x};  // u_hat + i (r_x)_hat, row a
        a = herm_ext(tileA + (G::P + p) * sh.C, e, M, sh.Kx);
        b = herm_ext(tileC + (G::P + p) * sh.C, e, M, sh.Kx);
        vb[m] = cd{a.x - b.y, a.y + b.x};  // row b
    }
    fft<M, true>(va, t, ex + p, G::P, tw);
    fft<M, true>(vb, t, ex + p, G::P, tw);
#pragma unroll
    for (int m = 0; m < 8; ++m) va[m] = cd{va[m].x * va[m].y, vb[m].x * vb[m].y};  // (u r_x)_a + i (u r_x)_b
    row_forward_store<M>(va, t, p, ex, tw, w.BD, g0, nrows, sh.C);
}

}  // namespace lo
