// Centre-symmetric loops (Sec. 3, eq. KS_loop_sym): a loop with u(-x, s) = -u(x, s) for every
// s is invariant under Xi, and the flow keeps it so. Every field of the step then has a fixed
// parity in x: u, u u_x, r and u r_x are odd, u_x and r_x even. An odd real field has a
// purely imaginary x-spectrum at every s (column j = 0 vanishes) and an even one a real
// x-spectrum, so one real number per (j, s) carries a column, and in s each column is the
// transform of a real sequence (Hermitian in k). State and intermediates halve.
//
// Per loop, with Kx the band edge in j and K1 = Ks + 1:
//   U, G  [j-1][k], j = 1..Kx, k = 0..Ks (complex): b_{j,k} = -i u_hat_{j,k}, Hermitian in k
//         (b_{j,-k} = conj b_{j,k}, b_{j,0} real); G holds U1 = b + dtau sigma G_lin;
//   A     [j-1][n] (real): Im u_j(s_n);    B then D: Im (u u_x)_j, Im (u r_x)_j;
//   C     [j-1][n] (real): (r_x)_j(s_n), which is real.
// In terms of b the residual, cost, period derivative and update take the forms of the full
// path (each term is linear in u_hat, so the factor -i passes through); the sums over the
// band run over j >= 1 (w_j = 2) and k >= 0, with k > 0 counted twice.
//
// Column transforms carry two columns j = 2c + 1, 2c + 2 in one complex transform
// (z = b_{2c+1}(s) + i b_{2c+2}(s)); row transforms are those of the full path on the odd and
// even half spectra.
#pragma once

#include "passes.hpp"

namespace lo {

struct XiWork {
    cd* U;
    cd* G;
    double* A;
    double* BD;
    double* Cb;
    double* partial;  // [l][j-1][2]
    double* J;
    double* dJdT;
    double* Told;
    int* status;
};

// ----------------------------------------------------------------------------- columns
struct XiColPos {
    bool active, two;  // two: the pair's second column exists (Kx may be odd)
    int l, j1, t, f;   // j1: 0-based index (j - 1) of the pair's first column
};

template <int N>
__device__ __forceinline__ XiColPos xi_col_pos(const Shape& sh, int block) {
    using G = ColG<N>;
    XiColPos p;
    p.t = threadIdx.x % G::TPF;
    p.f = threadIdx.x / G::TPF;
    const int NP = (sh.Kx + 1) / 2;
    const int gc = block * G::F + p.f;
    p.active = gc < sh.nloops * NP;
    p.l = p.active ? gc / NP : 0;
    p.j1 = p.active ? 2 * (gc % NP) : 0;
    p.two = p.active && p.j1 + 1 < sh.Kx;
    return p;
}

// Spectrum element e (FFT order) of z = b1 + i b2 from the half spectra c1 = b1_hat, c2 =
// b2_hat (k = 0..Ks) through Hermitian symmetry.
__device__ __forceinline__ cd xi_pack(const cd* c1, const cd* c2, int e, int N, int Ks, bool two) {
    if (e <= Ks) {
        const cd x = c1[e], y = two ? c2[e] : cd{0.0, 0.0};
        return cd{x.x - y.y, x.y + y.x};
    }
    if (e >= N - Ks) {
        const cd x = c1[N - e], y = two ? c2[N - e] : cd{0.0, 0.0};
        return cd{x.x + y.y, y.x - x.y};  // conj(x) + i conj(y)
    }
    return cd{0.0, 0.0};
}

// After a forward transform of z = b1 + i b2 (values v, thread t holding e = t + m TPF):
// the half spectra of b1 and b2, scaled by s, through the exchange region ex:
// b1_hat(e) = (Z_e + conj Z_{N-e}) / 2, b2_hat(e) = (Z_e - conj Z_{N-e}) / (2 i).
template <int N>
__device__ __forceinline__ void xi_split(const cd* v, int t, cd* ex, double s, cd* p1, cd* p2) {
    using G = ColG<N>;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) ex[xpos(t + m * G::TPF)] = v[m];
    xsync<G::TPF>();
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = t + m * G::TPF;
        const cd w = ex[xpos((N - e) & (N - 1))];
        const cd z = v[m];
        p1[m] = cd{0.5 * s * (z.x + w.x), 0.5 * s * (z.y - w.y)};
        p2[m] = cd{0.5 * s * (z.y + w.y), 0.5 * s * (w.x - z.x)};
    }
    xsync<G::TPF>();
}

// Hermitian extension in k of two half spectra held in registers (element e of g1, g2 at
// k = e <= Ks), through ex, into the inverse-transform input of z = b1 + i b2.
template <int N>
__device__ __forceinline__ void xi_extend(cd* v, const cd* g1, const cd* g2, int t, int Ks, bool two, cd* ex) {
    using G = ColG<N>;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = t + m * G::TPF;
        if (e <= Ks) {
            ex[xpos(2 * e)] = g1[m];
            ex[xpos(2 * e + 1)] = g2[m];
        }
    }
    xsync<G::TPF>();
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = t + m * G::TPF;
        cd z{0.0, 0.0};
        if (e <= Ks || e >= N - Ks) {
            const int k = e <= Ks ? e : N - e;
            const cd x = ex[xpos(2 * k)], y = two ? ex[xpos(2 * k + 1)] : cd{0.0, 0.0};
            z = e <= Ks ? cd{x.x - y.y, x.y + y.x} : cd{x.x + y.y, y.x - x.y};
        }
        v[m] = z;
    }
    xsync<G::TPF>();
}

template <int N>
__device__ __forceinline__ void xi_store_pair(const XiColPos& p, const Shape& sh, const cd* v, double* X) {
    using G = ColG<N>;
    if (!p.active) return;
    double* x1 = X + ((size_t)p.l * sh.Kx + p.j1) * N;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        x1[p.t + m * G::TPF] = v[m].x;
        if (p.two) x1[N + p.t + m * G::TPF] = v[m].y;
    }
}

template <int N>
__device__ __forceinline__ void xi_load_pair(const XiColPos& p, const Shape& sh, const double* X, cd* v) {
    using G = ColG<N>;
    const double* x1 = X + ((size_t)p.l * sh.Kx + p.j1) * N;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int n = p.t + m * G::TPF;
        v[m] = p.active ? cd{x1[n], p.two ? x1[N + n] : 0.0} : cd{0.0, 0.0};
    }
}

// Pass A: the inverse s-transforms of a pair of band columns into A.
template <int N>
__device__ __forceinline__ void xi_col_pass_A(const Shape& sh, int block, const XiWork& w, cd* ex,
                                              const cd* __restrict__ tw) {
    using G = ColG<N>;
    const XiColPos p = xi_col_pos<N>(sh, block);
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    const int K1 = sh.Ks + 1;
    const cd* b1 = w.U + ((size_t)p.l * sh.Kx + p.j1) * K1;
    cd v[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m)
        v[m] = p.active ? xi_pack(b1, b1 + K1, p.t + m * G::TPF, N, sh.Ks, p.two) : cd{0.0, 0.0};
    fft<N, G::PT, true>(v, p.t, ex + p.f * xlen<N>(), twc);
    xi_store_pair<N>(p, sh, v, w.A);
}

// Pass C: residual, the partial sums of J and dJ/dT, U1, and the inverse transform of r_x.
template <int N>
__device__ __forceinline__ void xi_col_pass_C(const Shape& sh, int block, const double* __restrict__ T,
                                              const XiWork& w, double dtau, int scheme, cd* ex, double* red,
                                              const cd* __restrict__ tw) {
    using G = ColG<N>;
    const XiColPos p = xi_col_pos<N>(sh, block);
    cd* exf = ex + p.f * xlen<N>();
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    cd v[G::PT];
    xi_load_pair<N>(p, sh, w.BD, v);
    fft<N, G::PT, false>(v, p.t, exf, twc);
    cd p1[G::PT], p2[G::PT];
    xi_split<N>(v, p.t, exf, 1.0 / N, p1, p2);

    const double Tl = p.active ? T[p.l] : 1.0;
    const double invT = 1.0 / Tl;
    const int K1 = sh.Ks + 1;
    double Jp[2] = {0.0, 0.0}, dTp[2] = {0.0, 0.0};
    cd g1[G::PT], g2[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        g1[m] = cd{0.0, 0.0};
        g2[m] = cd{0.0, 0.0};
        const int e = p.t + m * G::TPF;
        if (!p.active || e > sh.Ks) continue;
        const double om = kTwoPi * e;
        const double a = om * invT;
        const double wk = (e == 0) ? 2.0 : 4.0;  // w_j = 2 (j >= 1), k > 0 counted twice
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c == 1 && !p.two) break;
            const int jj = p.j1 + c;  // j - 1
            const double q = kTwoPi * (jj + 1) / sh.L;
            const double q2 = q * q, q4 = q2 * q2;
            const double lamx = -q4 * q4 + 2.0 * q4 * q2 - q4;
            const size_t at = ((size_t)p.l * sh.Kx + jj) * K1 + e;
            const cd b = w.U[at];
            const cd wh = c == 0 ? p1[m] : p2[m];
            // r = -(i om/T) b - (u u_x) + (q^2 - q^4) b in the b form
            cd r;
            r.x = a * b.y - wh.x + (q2 - q4) * b.x;
            r.y = -a * b.x - wh.y + (q2 - q4) * b.y;
            Jp[c] += wk * (r.x * r.x + r.y * r.y);
            dTp[c] += wk * om * (b.x * r.y - b.y * r.x);
            cd gl;
            gl.x = a * r.y + (q4 - q2) * r.x;
            gl.y = -a * r.x + (q4 - q2) * r.y;
            const double sig = scheme ? 1.0 / (1.0 - dtau * (lamx - a * a)) : 1.0;
            const double st = dtau * sig;
            w.G[at] = cd{b.x + st * gl.x, b.y + st * gl.y};  // U1
            const cd rx = cd{-q * r.x, -q * r.y};            // (r_x)_hat in the real-column form
            if (c == 0)
                g1[m] = rx;
            else
                g2[m] = rx;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double jp = Jp[c], tp = dTp[c];
        col_sum2<G::TPF>(jp, tp, red);
        if (p.active && p.t == 0 && (c == 0 || p.two)) {
            double* part = w.partial + ((size_t)p.l * sh.Kx + p.j1 + c) * 2;
            part[0] = jp;
            part[1] = tp;
        }
    }
    xi_extend<N>(v, g1, g2, p.t, sh.Ks, p.two, exf);
    fft<N, G::PT, true>(v, p.t, exf, twc);
    xi_store_pair<N>(p, sh, v, w.Cb);
}

// Pass E: the new state U1 - dtau sigma (u r_x)_hat, then the next step's A from it.
template <int N>
__device__ __forceinline__ void xi_col_pass_E(const Shape& sh, int block, const XiWork& w, double dtau, int scheme,
                                              bool fuseA, cd* ex, const cd* __restrict__ tw) {
    using G = ColG<N>;
    const XiColPos p = xi_col_pos<N>(sh, block);
    cd* exf = ex + p.f * xlen<N>();
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    cd v[G::PT];
    xi_load_pair<N>(p, sh, w.BD, v);
    fft<N, G::PT, false>(v, p.t, exf, twc);
    cd p1[G::PT], p2[G::PT];
    xi_split<N>(v, p.t, exf, 1.0 / N, p1, p2);
    const double Tl = p.active ? w.Told[p.l] : 1.0;
    const int K1 = sh.Ks + 1;
    cd g1[G::PT], g2[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        g1[m] = cd{0.0, 0.0};
        g2[m] = cd{0.0, 0.0};
        const int e = p.t + m * G::TPF;
        if (!p.active || e > sh.Ks) continue;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c == 1 && !p.two) break;
            const int jj = p.j1 + c;
            const double q = kTwoPi * (jj + 1) / sh.L;
            const double q2 = q * q, q4 = q2 * q2;
            const double lamx = -q4 * q4 + 2.0 * q4 * q2 - q4;
            double sig = 1.0;
            if (scheme) {
                const double a = kTwoPi * e / Tl;
                sig = 1.0 / (1.0 - dtau * (lamx - a * a));
            }
            const double st = dtau * sig;
            const size_t at = ((size_t)p.l * sh.Kx + jj) * K1 + e;
            const cd gg = w.G[at];
            const cd ph = c == 0 ? p1[m] : p2[m];
            const cd x = cd{gg.x - st * ph.x, gg.y - st * ph.y};
            w.U[at] = x;
            if (c == 0)
                g1[m] = x;
            else
                g2[m] = x;
        }
    }
    if (!fuseA) return;
    xi_extend<N>(v, g1, g2, p.t, sh.Ks, p.two, exf);
    fft<N, G::PT, true>(v, p.t, exf, twc);
    xi_store_pair<N>(p, sh, v, w.A);
}

// -------------------------------------------------------------------------------- rows
// Element e of the x-spectrum of an odd field (i b_j, j >= 1, conjugate for negative
// frequencies) and of an even field (real c_j), from real tiles [j-1][r].
__device__ __forceinline__ cd xi_herm_odd(const double* tile, int TS, int r, int e, int M, int Kx) {
    const int j = e <= M / 2 ? e : M - e;
    const bool in = j >= 1 && j <= Kx;
    const double v = tile[(in ? j - 1 : 0) * TS + r];
    return in ? cd{0.0, e <= M / 2 ? v : -v} : cd{0.0, 0.0};
}
__device__ __forceinline__ cd xi_herm_even(const double* tile, int TS, int r, int e, int M, int Kx) {
    const int j = e <= M / 2 ? e : M - e;
    const bool in = j >= 1 && j <= Kx;
    const double v = tile[(in ? j - 1 : 0) * TS + r];
    return in ? cd{v, 0.0} : cd{0.0, 0.0};
}

// Rows [g0, g0 + ROWS) of NT real intermediates into real tiles tile + q * TILE, [j-1][r].
template <int ROWS, int CMAX, int TS, int TILE, int NT>
__device__ __forceinline__ void xi_load_rows(double* tile, const double* const (&X)[NT], size_t g0, const Shape& sh,
                                             size_t nrows) {
    constexpr int NL = (ROWS * CMAX + kBlock - 1) / kBlock;
    const int n = ROWS * sh.Kx;
    double buf[NT][NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * kBlock;
        const int j = i / ROWS, r = i % ROWS;
        const size_t g = g0 + r;
        const bool ok = i < n && g < nrows;
        const size_t off = ok ? ((g >> sh.logN) * sh.Kx + j) * sh.N + (g & (size_t)(sh.N - 1)) : 0;
#pragma unroll
        for (int q = 0; q < NT; ++q) buf[q][k] = ok ? X[q][off] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * kBlock;
        if (i < n) {
            const int j = i / ROWS, r = i % ROWS;
#pragma unroll
            for (int q = 0; q < NT; ++q) tile[q * TILE + j * TS + r] = buf[q][k];
        }
    }
}

// The imaginary parts of the output tile (an odd product: its real parts vanish) for
// j = 1..Kx into the real intermediate X.
template <int ROWS, int CMAX>
__device__ __forceinline__ void xi_store_rows(const cd* tile, int TS, double* X, size_t g0, const Shape& sh,
                                              size_t nrows) {
    constexpr int NL = (ROWS * CMAX + kBlock - 1) / kBlock;
    const int n = ROWS * sh.Kx;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * kBlock;
        const int j = i / ROWS, r = i % ROWS;
        const size_t g = g0 + r;
        if (i < n && g < nrows)
            X[((g >> sh.logN) * sh.Kx + j) * sh.N + (g & (size_t)(sh.N - 1))] = tile[(j + 1) * TS + r].y;
    }
}

template <int M>
__device__ __forceinline__ void xi_row_pass_B(const Shape& sh, int block, const XiWork& w, cd* lds,
                                              const cd* __restrict__ tw) {
    using G = RowG<M>;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const size_t g0 = (size_t)block * G::ROWS;
    const int t = threadIdx.x % G::TPF, p = threadIdx.x / G::TPF;
    TwCache<M, G::PT> twc;
    tw_cache_load<M, G::PT>(twc, t, tw);
    double* tl = reinterpret_cast<double*>(lds);
    {
        const double* const src[1] = {w.A};
        xi_load_rows<G::ROWS, G::CMAX, G::TS, G::TILE, 1>(tl, src, g0, sh, nrows);
    }
    __syncthreads();
    const double dq = kTwoPi / sh.L;
    cd va[G::PT], vb[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = t + m * G::TPF;
        const double q = dq * (double)((e <= M / 2) ? e : e - M);
        const cd a = xi_herm_odd(tl, G::TS, p, e, M, sh.Kx), b = xi_herm_odd(tl, G::TS, G::P + p, e, M, sh.Kx);
        va[m] = pack2(a, b);
        vb[m] = pack2(cd{-q * a.y, q * a.x}, cd{-q * b.y, q * b.x});
    }
    row_products<M>(sh, va, vb, lds, t, p, twc);
    xi_store_rows<G::ROWS, G::CMAX>(lds, G::TS, w.BD, g0, sh, nrows);
}

template <int M>
__device__ __forceinline__ void xi_row_pass_D(const Shape& sh, int block, const XiWork& w, double* T,
                                              double dtau, double* J_hist, cd* lds, const cd* __restrict__ tw) {
    using G = RowG<M>;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const size_t g0 = (size_t)block * G::ROWS;
    const int t = threadIdx.x % G::TPF, p = threadIdx.x / G::TPF;
    TwCache<M, G::PT> twc;
    tw_cache_load<M, G::PT>(twc, t, tw);
    double* tA = reinterpret_cast<double*>(lds);
    double* tC = tA + G::TILE;
    {
        const double* const src[2] = {w.A, w.Cb};
        xi_load_rows<G::ROWS, G::CMAX, G::TS, G::TILE, 2>(tA, src, g0, sh, nrows);
    }
    // loops whose first row lies in this block are finished here (partials from pass C)
    if (threadIdx.x < 64) {
        Shape sx = sh;
        sx.C = sh.Kx;  // one partial pair per column j = 1..Kx
        Work wf{};
        wf.partial = w.partial;
        wf.J = w.J;
        wf.dJdT = w.dJdT;
        wf.Told = w.Told;
        wf.status = w.status;
        const size_t l0 = (g0 + sh.N - 1) >> sh.logN;
        for (size_t l = l0; (l << sh.logN) < g0 + G::ROWS && l < (size_t)sh.nloops; ++l)
            finalize_loop(sx, (int)l, wf, T, MODE_STEP, dtau, J_hist, nullptr, nullptr);
    }
    __syncthreads();
    cd va[G::PT], vb[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = t + m * G::TPF;
        va[m] = pack2(xi_herm_odd(tA, G::TS, p, e, M, sh.Kx), xi_herm_odd(tA, G::TS, G::P + p, e, M, sh.Kx));
        vb[m] = pack2(xi_herm_even(tC, G::TS, p, e, M, sh.Kx), xi_herm_even(tC, G::TS, G::P + p, e, M, sh.Kx));
    }
    row_products<M>(sh, va, vb, lds, t, p, twc);
    xi_store_rows<G::ROWS, G::CMAX>(lds, G::TS, w.BD, g0, sh, nrows);
}

}  // namespace lo
