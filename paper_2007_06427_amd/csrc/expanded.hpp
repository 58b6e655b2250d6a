// The paper's own evaluation of the flow (Sec. 4.2, eq. KS_G_1), as a cross-check of the
// residual-then-adjoint passes and as the paper's step:
//   G_1L  = (1/T^2) u_ss - u_xxxxxxxx - 2 u_xxxxxx - u_xxxx        (lambda u_hat in the band),
//   G_1NL = -5 u_xxxx u_x - 10 u_xxx u_xx - 3 u_xx u_x + u^2 u_xx + u u_x^2
//           + (2u/T) u_xs + (1/T) u_x u_s,
// with derivatives in spectral space, the fields on the grid, the products pointwise there
// and G_1NL transformed back and truncated to the band. dJ/dT = int int (1/T^2) u_s r and
// J = 1/2 int int r^2 take their integrands on the grid, r = -(1/T) u_s - u u_x - u_xx - u_xxxx
// formed pointwise (the (0, 0) mode times L).
//
// Three passes instead of five: one row pass forms every product at once.
//   XA (columns): inverse s-transforms of u_hat_j and (i omega) u_hat_j  -> A, Cb
//   XB (rows):    seven inverse x-transforms (u, u_x .. u_xxxx from A; u_s, u_xs from Cb), the
//                 pointwise G_1NL, r, and per-row sums of r^2 and u_s r, then one forward
//                 transform of G_1NL -> BD (columns j <= Kx)
//   finalize:     per loop, J and dJ/dT from the row sums (and T's update when stepping)
//   XC (columns): forward s-transform of BD: G_1 = lambda u_hat + G_1NL_hat, or the update
//                 u_hat' = (u_hat + dtau G_1NL_hat) / (1 - dtau lambda) (IMEX) or
//                 u_hat + dtau G_1 (explicit); optionally XA of the next step.
// The per-row sums live in the band buffer G (two doubles per row; G holds no band values
// until XC), already scaled by 1/(Nx Ns), so that the per-loop sum uses finalize_loop.
#pragma once

#include "passes.hpp"

namespace lo {

// A and Cb from band column values v (zero outside the band): IFFT of v and of (i omega) v.
template <int N>
__device__ __forceinline__ void x_inverse_pair(const Shape& sh, const ColPos& p, const cd* v, const Work& w, cd* ex,
                                               const TwCache<N, ColG<N>::PT>& twc) {
    using G = ColG<N>;
    cd a[G::PT], b[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = p.t + m * G::TPF;
        const double om = kTwoPi * (double)((e < N / 2) ? e : e - N);
        a[m] = v[m];
        b[m] = cd{-om * v[m].y, om * v[m].x};
    }
    col_inverse_store<N>(sh, p, a, w.A, ex, twc);
    col_inverse_store<N>(sh, p, b, w.Cb, ex, twc);
}

template <int N>
__device__ __forceinline__ void col_pass_XA(const Shape& sh, int block, const Work& w, cd* ex,
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
        v[m] = (p.active && kk >= 0) ? u[kk] : cd{0.0, 0.0};
    }
    x_inverse_pair<N>(sh, p, v, w, ex, twc);
}

// Tl: the period at the start of the step (Told when stepping, T otherwise).
template <int N>
__device__ __forceinline__ void col_pass_XC(const Shape& sh, int block, const Work& w, const double* __restrict__ Tl_,
                                            int mode, double dtau, int scheme, bool fuse, cd* ex,
                                            const cd* __restrict__ tw) {
    using G = ColG<N>;
    const ColPos p = col_pos<N>(sh, block);
    const size_t col = (size_t)p.l * sh.C + p.j;
    const cd* Xc = w.BD + col * N;
    cd v[G::PT];
#pragma unroll
    for (int m = 0; m < G::PT; ++m) v[m] = p.active ? Xc[p.t + m * G::TPF] : cd{0.0, 0.0};
    TwCache<N, G::PT> twc;
    tw_cache_load<N, G::PT>(twc, p.t, tw);
    fft<N, G::PT, false>(v, p.t, ex + p.f * xlen<N>(), twc);
    const double Tl = p.active ? Tl_[p.l] : 1.0;
    const double q = kTwoPi * p.j / sh.L;
    const double q2 = q * q, q4 = q2 * q2;
    const double lamx = -q4 * q4 + 2.0 * q4 * q2 - q4;
    const double invN = 1.0 / N;
    cd* u = w.U + col * sh.NB;
    cd* g = w.G + col * sh.NB;
#pragma unroll
    for (int m = 0; m < G::PT; ++m) {
        const int e = p.t + m * G::TPF;
        const int kk = band_row(e, N, sh.Ks);
        cd x{0.0, 0.0};
        if (p.active && kk >= 0) {
            const double a = kTwoPi * (double)((e < N / 2) ? e : e - N) / Tl;
            const double lm = lamx - a * a;
            const cd nl = cscale(v[m], invN);
            const cd uu = u[kk];
            if (mode == MODE_STEP) {
                if (scheme) {
                    const double d = 1.0 / (1.0 - dtau * lm);
                    x = cd{(uu.x + dtau * nl.x) * d, (uu.y + dtau * nl.y) * d};
                } else {
                    x = cd{uu.x + dtau * (lm * uu.x + nl.x), uu.y + dtau * (lm * uu.y + nl.y)};
                }
                u[kk] = x;
            } else {
                g[kk] = cd{lm * uu.x + nl.x, lm * uu.y + nl.y};
            }
        }
        v[m] = x;
    }
    if (fuse) x_inverse_pair<N>(sh, p, v, w, ex, twc);
}

// LDS of the row pass: the A and Cb tiles stay readable while the exchange regions (after
// them) carry the transforms.
template <int M>
struct XRowG {
    using G = RowG<M>;
    static constexpr int EX = 2 * G::TILE;
    static constexpr int LDS = 2 * G::TILE + G::XL;  // complex values
};

// (i q)^n z for n = 0 .. 4
__device__ __forceinline__ cd ipow_q(cd z, double q, int n) {
    const double q2 = q * q;
    switch (n) {
        case 0: return z;
        case 1: return cd{-q * z.y, q * z.x};
        case 2: return cd{-q2 * z.x, -q2 * z.y};
        case 3: return cd{q2 * q * z.y, -q2 * q * z.x};
        default: return cd{q2 * q2 * z.x, q2 * q2 * z.y};
    }
}

template <int M>
__device__ __forceinline__ void row_pass_X(const Shape& sh, int block, const Work& w, const double* __restrict__ T,
                                           cd* lds, const cd* __restrict__ tw) {
    using G = RowG<M>;
    constexpr int PT = G::PT;
    const size_t nrows = (size_t)sh.nloops * sh.N;
    const size_t g0 = (size_t)block * G::ROWS;
    const int t = threadIdx.x % G::TPF, p = threadIdx.x / G::TPF;
    TwCache<M, PT> twc;
    tw_cache_load<M, PT>(twc, t, tw);
    cd* tA = lds;
    cd* tS = lds + G::TILE;
    cd* ex = lds + XRowG<M>::EX + p * xlen<M>();
    {
        const cd* const src[2] = {w.A, w.Cb};
        load_rows<G::ROWS, G::CMAX, G::TS, G::TILE, 2>(tA, src, g0, sh, nrows);
    }
    __syncthreads();
    const size_t ga = g0 + p, gb = g0 + G::P + p;
    const double ia = ga < nrows ? 1.0 / T[ga >> sh.logN] : 1.0;
    const double ib = gb < nrows ? 1.0 / T[gb >> sh.logN] : 1.0;
    const double dq = kTwoPi / sh.L;
    // values of the field (i q)^n X on rows a (real parts) and b (imaginary parts)
    auto field = [&](const cd* tile, int n, cd* v) {
#pragma unroll
        for (int m = 0; m < PT; ++m) {
            const int e = t + m * G::TPF;
            const double q = dq * (double)((e <= M / 2) ? e : e - M);
            const cd a = herm_ext(tile, G::TS, p, e, M, sh.Kx), b = herm_ext(tile, G::TS, G::P + p, e, M, sh.Kx);
            v[m] = pack2(ipow_q(a, q, n), ipow_q(b, q, n));
        }
        fft<M, PT, true>(v, t, ex, twc);
    };
    cd u[PT], u1[PT], u2[PT], f[PT], acc[PT], r[PT];
    field(tA, 0, u);
    field(tA, 1, u1);
    field(tA, 2, u2);
    field(tA, 3, f);  // u_xxx
#pragma unroll
    for (int m = 0; m < PT; ++m) acc[m] = cd{-10.0 * f[m].x * u2[m].x, -10.0 * f[m].y * u2[m].y};
    field(tA, 4, f);  // u_xxxx
#pragma unroll
    for (int m = 0; m < PT; ++m) {
        acc[m].x += -5.0 * f[m].x * u1[m].x;
        acc[m].y += -5.0 * f[m].y * u1[m].y;
        r[m] = cd{-u[m].x * u1[m].x - u2[m].x - f[m].x, -u[m].y * u1[m].y - u2[m].y - f[m].y};
    }
    field(tS, 0, f);  // u_s
    double ja = 0.0, jb = 0.0, da = 0.0, db = 0.0;
#pragma unroll
    for (int m = 0; m < PT; ++m) {
        acc[m].x += ia * u1[m].x * f[m].x;
        acc[m].y += ib * u1[m].y * f[m].y;
        r[m].x += -ia * f[m].x;
        r[m].y += -ib * f[m].y;
        ja += r[m].x * r[m].x;
        jb += r[m].y * r[m].y;
        da += f[m].x * r[m].x;
        db += f[m].y * r[m].y;
    }
    field(tS, 1, f);  // u_xs
#pragma unroll
    for (int m = 0; m < PT; ++m) {
        acc[m].x += 2.0 * ia * u[m].x * f[m].x - 3.0 * u2[m].x * u1[m].x + u[m].x * u[m].x * u2[m].x +
                    u[m].x * u1[m].x * u1[m].x;
        acc[m].y += 2.0 * ib * u[m].y * f[m].y - 3.0 * u2[m].y * u1[m].y + u[m].y * u[m].y * u2[m].y +
                    u[m].y * u1[m].y * u1[m].y;
    }
    // per-row sums over x, scaled by 1/(M N): finalize_loop then forms J and dJ/dT
    ja = wsum_lanes(ja, G::TPF);
    jb = wsum_lanes(jb, G::TPF);
    da = wsum_lanes(da, G::TPF);
    db = wsum_lanes(db, G::TPF);
    if (t == 0) {
        const double s = 1.0 / ((double)M * sh.N);
        double* part = reinterpret_cast<double*>(w.G);
        if (ga < nrows) {
            part[2 * ga] = ja * s;
            part[2 * ga + 1] = da * s;
        }
        if (gb < nrows) {
            part[2 * gb] = jb * s;
            part[2 * gb + 1] = db * s;
        }
    }
    // forward transform of G_1NL (rows a + i b), split into the two rows' half spectra
    fft<M, PT, false>(acc, t, ex, twc);
#pragma unroll
    for (int m = 0; m < PT; ++m) ex[xpos(t + m * G::TPF)] = acc[m];
    wave_lds_order();
    const int lane = threadIdx.x % 64;
    const int pw0 = (threadIdx.x / 64) * G::PW;
    const int nout = 2 * G::PW * sh.C;
    const double s = 0.5 / M;
    cd outv[G::NOUT];
#pragma unroll
    for (int i = 0; i < G::NOUT; ++i) {
        const int idx = lane + 64 * i;
        if (idx < nout) {
            const int pp = pw0 + idx / (2 * sh.C);
            const int rem = idx % (2 * sh.C);
            const int j = rem % sh.C;
            const cd* e2 = lds + XRowG<M>::EX + pp * xlen<M>();
            const cd a = e2[xpos(j)];
            const cd b = e2[xpos((M - j) & (M - 1))];
            outv[i] = rem >= sh.C ? cd{(a.y + b.y) * s, (b.x - a.x) * s} : cd{(a.x + b.x) * s, (a.y - b.y) * s};
        }
    }
    __syncthreads();  // every wave is done with the input tiles: the output tile overwrites tA
#pragma unroll
    for (int i = 0; i < G::NOUT; ++i) {
        const int idx = lane + 64 * i;
        if (idx < nout) {
            const int pp = pw0 + idx / (2 * sh.C);
            const int rem = idx % (2 * sh.C);
            // consecutive lanes write consecutive j of one row (row b after row a)
            lds[(rem % sh.C) * G::TS + (rem >= sh.C ? G::P + pp : pp)] = outv[i];
        }
    }
    __syncthreads();
    store_rows<G::ROWS, G::CMAX>(lds, G::TS, w.BD, g0, sh, nrows);
}

}  // namespace lo
