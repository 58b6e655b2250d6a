// liblooporbit: C ABI and kernels for the fictitious-time step of the KS loop dynamics
// (Azimi, Ashtari & Schneider, arXiv:2007.06427, Sec. 3-4). See include/looporbit.h for the
// contract of each entry point and passes.hpp for the pass decomposition.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <string>
#include <mutex>
#include <type_traits>
#include <vector>

#include "looporbit.h"
#include "passes.hpp"
#include "resident.hpp"
#include "xi.hpp"
#include "expanded.hpp"

using namespace lo;

// Work space of loop_step_noalloc, for callers that cannot allocate: one copy per device, held
// from the library's load until the process ends. Host code never uses this name as an
// address (on the host it is only a handle): it takes each device's address from
// hipGetSymbolAddress once (init_scratch) and passes that pointer to the kernels.
constexpr size_t kScratchBytes = LOOP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// ============================================================================ kernels
template <int N>
__global__ __launch_bounds__(kBlock) void k_colA(Shape sh, Work w, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    col_pass_A<N>(sh, blockIdx.x, w, ex, tw);
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_rowB(Shape sh, Work w, const cd* __restrict__ tw) {
    __shared__ cd lds[RowG<M>::LDS_B];
    row_pass_B<M>(sh, blockIdx.x, w, lds, tw);
}

// The column kernels are compiled per mode, so that each allocates registers for its own
// work only (the residual-only forward has no inverse transform).
template <int N, int MODE>
__global__ __launch_bounds__(kBlock) void k_colC(Shape sh, const double* __restrict__ T, Work w, double dtau,
                                                 int scheme, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    __shared__ double red[2 * kBlock / 64];
    col_pass_C<N>(sh, blockIdx.x, T, w, MODE, dtau, scheme, ex, red, tw);
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_rowD(Shape sh, Work w, double* T, int mode, double dtau,
                                                 double* J_hist, double* Jout, double* dJdTout,
                                                 const cd* __restrict__ tw) {
    __shared__ cd lds[RowG<M>::LDS];
    row_pass_D<M>(sh, blockIdx.x, w, T, mode, dtau, J_hist, Jout, dJdTout, lds, tw);
}

template <int N, int MODE>
__global__ __launch_bounds__(kBlock) void k_colE(Shape sh, Work w, double dtau, int scheme, int fuseA,
                                                 const cd* __restrict__ tw, const double* __restrict__ T) {
    __shared__ cd ex[ColG<N>::LDS];
    col_pass_E<N>(sh, blockIdx.x, w, MODE, dtau, scheme, fuseA != 0, ex, tw, T);
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_colAC(Shape sh, Work w, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    col_pass_AC<N>(sh, blockIdx.x, w, ex, tw);
}

// the residual half of k_colAC, for a reverse pass given u on the s grid
template <int N>
__global__ __launch_bounds__(kBlock) void k_colR(Shape sh, Work w, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    col_pass_AC<N, false>(sh, blockIdx.x, w, ex, tw);
}

// one wavefront per loop
__global__ __launch_bounds__(64) void k_finalize(Shape sh, Work w, double* T, double* Jout, double* dJdTout) {
    finalize_loop(sh, blockIdx.x, w, T, MODE_COST, 0.0, nullptr, Jout, dJdTout);
}

// The paper's expanded form of the flow (expanded.hpp): three passes and a per-loop finalize.
template <int N>
__global__ __launch_bounds__(kBlock) void k_xA(Shape sh, Work w, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    col_pass_XA<N>(sh, blockIdx.x, w, ex, tw);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_xB(Shape sh, Work w, const double* __restrict__ T,
                                               const cd* __restrict__ tw) {
    extern __shared__ __align__(16) cd lds[];  // 16-byte aligned: one ds_read_b128 per complex value
    row_pass_X<M>(sh, blockIdx.x, w, T, lds, tw);
}
// one wavefront per loop: the row sums (in G) of loop blockIdx.x into J, dJ/dT (and T's update)
__global__ __launch_bounds__(64) void k_x_finalize(Shape sh, Work w, double* T, int mode, double dtau,
                                                   double* J_hist, double* Jout, double* dJdTout) {
    Shape sx = sh;
    sx.C = sh.N;  // one partial pair per row
    Work wf = w;
    wf.partial = reinterpret_cast<double*>(w.G);
    finalize_loop(sx, blockIdx.x, wf, T, mode, dtau, J_hist, Jout, dJdTout);
}
template <int N>
__global__ __launch_bounds__(kBlock) void k_xC(Shape sh, Work w, const double* __restrict__ Tl, int mode, double dtau,
                                               int scheme, int fuse, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    col_pass_XC<N>(sh, blockIdx.x, w, Tl, mode, dtau, scheme, fuse != 0, ex, tw);
}

// Centre-symmetric form (xi.hpp): one pass per kernel over all loops of one shape.
template <int N>
__global__ __launch_bounds__(kBlock) void k_xi_colA(Shape sh, XiWork w, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    xi_col_pass_A<N>(sh, blockIdx.x, w, ex, tw);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_xi_rowB(Shape sh, XiWork w, const cd* __restrict__ tw) {
    __shared__ cd lds[RowG<M>::LDS];
    xi_row_pass_B<M>(sh, blockIdx.x, w, lds, tw);
}
template <int N>
__global__ __launch_bounds__(kBlock) void k_xi_colC(Shape sh, const double* __restrict__ T, XiWork w, double dtau,
                                                    int scheme, const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    __shared__ double red[2 * kBlock / 64];
    xi_col_pass_C<N>(sh, blockIdx.x, T, w, dtau, scheme, ex, red, tw);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_xi_rowD(Shape sh, XiWork w, double* T, double dtau, double* J_hist,
                                                    const cd* __restrict__ tw) {
    __shared__ cd lds[RowG<M>::LDS];
    xi_row_pass_D<M>(sh, blockIdx.x, w, T, dtau, J_hist, lds, tw);
}
template <int N>
__global__ __launch_bounds__(kBlock) void k_xi_colE(Shape sh, XiWork w, double dtau, int scheme, int fuseA,
                                                    const cd* __restrict__ tw) {
    __shared__ cd ex[ColG<N>::LDS];
    xi_col_pass_E<N>(sh, blockIdx.x, w, dtau, scheme, fuseA != 0, ex, tw);
}

// rfft layout -> centre-symmetric band state, projecting orthogonally onto centre-symmetric
// loops: u_hat_{j,k} -> (u_hat_{j,k} - conj u_hat_{j,-k}) / 2, stored as b = -i u_hat (k >= 0).
__global__ __launch_bounds__(256) void k_to_xi(Shape sh, const cd* __restrict__ uhat, cd* __restrict__ U) {
    const int K1 = sh.Ks + 1;
    const size_t total = (size_t)sh.nloops * sh.Kx * K1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % K1);
        const size_t lj = i / K1;
        const int j = (int)(lj % sh.Kx) + 1;
        const size_t l = lj / sh.Kx;
        const cd* u = uhat + l * sh.N * sh.H;
        const cd a = u[(size_t)k * sh.H + j];
        const cd b = u[(size_t)((sh.N - k) & (sh.N - 1)) * sh.H + j];
        const cd d = cd{a.x - b.x, a.y + b.y};  // u_{j,k} - conj u_{j,-k}
        U[i] = cd{0.5 * d.y, -0.5 * d.x};
    }
}

// centre-symmetric band state -> rfft layout, every entry written (0 outside the band):
// u_hat_{j,k} = i b_{j,k}, u_hat_{j,-k} = i conj b_{j,k}.
__global__ __launch_bounds__(256) void k_from_xi(Shape sh, const cd* __restrict__ U, cd* __restrict__ out) {
    const int K1 = sh.Ks + 1;
    const size_t total = (size_t)sh.nloops * sh.N * sh.H;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % sh.H);
        const size_t le = i / sh.H;
        const int e = (int)(le % sh.N);
        const size_t l = le / sh.N;
        cd v{0.0, 0.0};
        if (j >= 1 && j <= sh.Kx) {
            const cd* b = U + (l * sh.Kx + (j - 1)) * K1;
            if (e <= sh.Ks) {
                const cd x = b[e];
                v = cd{-x.y, x.x};
            } else if (e >= sh.N - sh.Ks) {
                const cd x = b[sh.N - e];
                v = cd{x.y, x.x};
            }
        }
        out[i] = v;
    }
}

// rfft layout -> band layout U[l][j][kk], column 0 through its Hermitian part (32 x 32 tiles).
__global__ __launch_bounds__(256) void k_to_band(Shape sh, const cd* __restrict__ uhat, cd* __restrict__ U) {
    __shared__ cd tile[32][33];
    const int l = blockIdx.z, kk0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty0 = threadIdx.x / 32;
    const cd* u = uhat + (size_t)l * sh.N * sh.H;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int kk = kk0 + ty, j = j0 + tx;
        cd v{0.0, 0.0};
        if (kk < sh.NB && j < sh.C) {
            const int e = (kk <= sh.Ks) ? kk : kk + sh.N - sh.NB;
            v = u[(size_t)e * sh.H + j];
            if (j == 0) {
                const cd pr = u[(size_t)((sh.N - e) & (sh.N - 1)) * sh.H];
                v = cd{0.5 * (v.x + pr.x), 0.5 * (v.y - pr.y)};
            }
        }
        tile[ty][tx] = v;
    }
    __syncthreads();
    cd* dst = U + (size_t)l * sh.C * sh.NB;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int j = j0 + ty, kk = kk0 + tx;
        if (j < sh.C && kk < sh.NB) dst[(size_t)j * sh.NB + kk] = tile[tx][ty];
    }
}

// band layout [l][j][kk] -> rfft layout, every entry written (0 outside the band).
__global__ __launch_bounds__(256) void k_from_band(Shape sh, const cd* __restrict__ src, cd* __restrict__ out) {
    __shared__ cd tile[32][33];
    const int l = blockIdx.z, e0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty0 = threadIdx.x / 32;
    const cd* s = src + (size_t)l * sh.C * sh.NB;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int j = j0 + ty, e = e0 + tx;
        // a select of the loaded value (a local assigned in a branch would live in scratch)
        const int kk = (j < sh.C && e < sh.N) ? band_row(e, sh.N, sh.Ks) : -1;
        tile[ty][tx] = kk >= 0 ? s[(size_t)j * sh.NB + kk] : cd{0.0, 0.0};
    }
    __syncthreads();
    cd* o = out + (size_t)l * sh.N * sh.H;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int e = e0 + ty, j = j0 + tx;
        if (e < sh.N && j < sh.H) o[(size_t)e * sh.H + j] = tile[tx][ty];
    }
}

// Gradient of sum_l gJ[l] J_l in torch's complex convention (d/dRe + i d/dIm) from G_1 in
// band layout: grad[l][e][j] = -gJ[l] w_j L G_1, with w_0 = 1 and w_j = 2 for j >= 1. A
// coefficient with j >= 1 stands for itself and its partner (-j, -k); column 0 holds both
// partners. Every entry of the output is written, 0 outside the band.
__global__ __launch_bounds__(256) void k_grad_from_band(Shape sh, const cd* __restrict__ src, const double* gJ,
                                                        cd* __restrict__ out) {
    __shared__ cd tile[32][33];
    const int l = blockIdx.z, e0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty0 = threadIdx.x / 32;
    const cd* s = src + (size_t)l * sh.C * sh.NB;
    const double g = (gJ ? gJ[l] : 1.0) * sh.L;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int j = j0 + ty, e = e0 + tx;
        cd v{0.0, 0.0};
        if (j < sh.C && e < sh.N) {
            const int kk = band_row(e, sh.N, sh.Ks);
            if (kk >= 0) {
                const double f = -g * (j == 0 ? 1.0 : 2.0);
                const cd x = s[(size_t)j * sh.NB + kk];
                v = cd{f * x.x, f * x.y};
            }
        }
        tile[ty][tx] = v;
    }
    __syncthreads();
    cd* o = out + (size_t)l * sh.N * sh.H;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int e = e0 + ty, j = j0 + tx;
        if (e < sh.N && j < sh.H) o[(size_t)e * sh.H + j] = tile[tx][ty];
    }
}

__global__ void k_grad_T(int nloops, const double* gJ, const double* __restrict__ dJdT, double* gradT) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nloops) gradT[l] = (gJ ? gJ[l] : 1.0) * dJdT[l];
}

// uhat <- canonical(uhat) + dtau * sigma * Hermitian-part(Ghat) in the band, 0 outside (rfft layout).
__global__ void k_update(Shape sh, const double* __restrict__ T, cd* uhat, const cd* __restrict__ Ghat,
                         double dtau, int scheme) {
    const size_t per = (size_t)sh.N * sh.H;
    const size_t total = per * sh.nloops;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t l = i / per;
        const int e = (int)((i % per) / sh.H), j = (int)(i % sh.H);
        if (j == 0 && e > sh.N / 2) continue;  // handled with its partner row
        cd* u = uhat + l * per;
        const cd* g = Ghat + l * per;
        const bool inb = band_row(e, sh.N, sh.Ks) >= 0 && j < sh.C;
        const int e2 = (sh.N - e) & (sh.N - 1);
        if (!inb) {
            u[(size_t)e * sh.H + j] = cd{0.0, 0.0};
            if (j == 0) u[(size_t)e2 * sh.H] = cd{0.0, 0.0};
            continue;
        }
        cd uu = u[(size_t)e * sh.H + j], gg = g[(size_t)e * sh.H + j];
        if (j == 0) {
            const cd pu = u[(size_t)e2 * sh.H], pg = g[(size_t)e2 * sh.H];
            uu = cd{0.5 * (uu.x + pu.x), 0.5 * (uu.y - pu.y)};
            gg = cd{0.5 * (gg.x + pg.x), 0.5 * (gg.y - pg.y)};
        }
        double sig = 1.0;
        if (scheme == 1) {
            const int k = (e < sh.N / 2) ? e : e - sh.N;
            const double q = kTwoPi * j / sh.L, q2 = q * q, q4 = q2 * q2;
            const double a = kTwoPi * k / T[l];
            sig = 1.0 / (1.0 - dtau * (-q4 * q4 + 2.0 * q4 * q2 - q4 - a * a));
        }
        const double s = dtau * sig;
        const cd v{uu.x + s * gg.x, uu.y + s * gg.y};
        u[(size_t)e * sh.H + j] = v;
        if (j == 0) u[(size_t)e2 * sh.H] = cconj(v);
    }
}

// The update from a gradient in torch's convention (the gradient of sum_l J_l): G_1 = -grad /
// (w_j L), then as k_update. rfft layout.
__global__ void k_update_grad(Shape sh, const double* __restrict__ T, cd* uhat, const cd* __restrict__ grad,
                              double dtau, int scheme) {
    const size_t per = (size_t)sh.N * sh.H;
    const size_t total = per * sh.nloops;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t l = i / per;
        const int e = (int)((i % per) / sh.H), j = (int)(i % sh.H);
        if (j == 0 && e > sh.N / 2) continue;  // handled with its partner row
        cd* u = uhat + l * per;
        const cd* g = grad + l * per;
        const bool inb = band_row(e, sh.N, sh.Ks) >= 0 && j < sh.C;
        const int e2 = (sh.N - e) & (sh.N - 1);
        if (!inb) {
            u[(size_t)e * sh.H + j] = cd{0.0, 0.0};
            if (j == 0) u[(size_t)e2 * sh.H] = cd{0.0, 0.0};
            continue;
        }
        cd uu = u[(size_t)e * sh.H + j], gg = g[(size_t)e * sh.H + j];
        if (j == 0) {
            const cd pu = u[(size_t)e2 * sh.H], pg = g[(size_t)e2 * sh.H];
            uu = cd{0.5 * (uu.x + pu.x), 0.5 * (uu.y - pu.y)};
            gg = cd{0.5 * (gg.x + pg.x), 0.5 * (gg.y - pg.y)};
        }
        const double f = -1.0 / ((j == 0 ? 1.0 : 2.0) * sh.L);  // G_1 = -grad / (w_j L)
        gg = cd{f * gg.x, f * gg.y};
        double sig = 1.0;
        if (scheme == 1) {
            const int k = (e < sh.N / 2) ? e : e - sh.N;
            const double q = kTwoPi * j / sh.L, q2 = q * q, q4 = q2 * q2;
            const double a = kTwoPi * k / T[l];
            sig = 1.0 / (1.0 - dtau * (-q4 * q4 + 2.0 * q4 * q2 - q4 - a * a));
        }
        const double s = dtau * sig;
        const cd v{uu.x + s * gg.x, uu.y + s * gg.y};
        u[(size_t)e * sh.H + j] = v;
        if (j == 0) u[(size_t)e2 * sh.H] = cconj(v);
    }
}

// The same update on band-layout state and gradient ([l][j][kk]); column 0 is read through its
// Hermitian part and written Hermitian (one thread per pair k, -k).
__global__ void k_update_grad_band(Shape sh, const double* __restrict__ T, cd* ub, const cd* __restrict__ grad,
                                   double dtau, int scheme) {
    const size_t per = (size_t)sh.C * sh.NB;
    const size_t total = per * sh.nloops;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t l = i / per;
        const int j = (int)((i % per) / sh.NB), kk = (int)(i % sh.NB);
        if (j == 0 && kk > sh.Ks) continue;  // handled with its partner
        cd* u = ub + l * per + (size_t)j * sh.NB;
        const cd* g = grad + l * per + (size_t)j * sh.NB;
        const int kp = band_partner(kk, sh.NB);
        cd uu = u[kk], gg = g[kk];
        if (j == 0) {
            const cd pu = u[kp], pg = g[kp];
            uu = cd{0.5 * (uu.x + pu.x), 0.5 * (uu.y - pu.y)};
            gg = cd{0.5 * (gg.x + pg.x), 0.5 * (gg.y - pg.y)};
        }
        const double f = -1.0 / ((j == 0 ? 1.0 : 2.0) * sh.L);
        gg = cd{f * gg.x, f * gg.y};
        double sig = 1.0;
        if (scheme == 1) {
            const int k = (kk <= sh.Ks) ? kk : kk - sh.NB;
            const double q = kTwoPi * j / sh.L, q2 = q * q, q4 = q2 * q2;
            const double a = kTwoPi * k / T[l];
            sig = 1.0 / (1.0 - dtau * (-q4 * q4 + 2.0 * q4 * q2 - q4 - a * a));
        }
        const double s = dtau * sig;
        const cd v{uu.x + s * gg.x, uu.y + s * gg.y};
        u[kk] = v;
        if (j == 0 && kk != 0) u[kp] = cconj(v);
    }
}

__global__ void k_update_T(int nloops, double* T, const double* __restrict__ dJdT, double dtau) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nloops) T[l] = T[l] - dtau * dJdT[l];
}

// Linear extrapolation of whole loops along their trajectory (App. C):
// l <- l + f[l] (l - l_a) for l = (u_hat in rfft layout, T); f = 0 leaves a loop unchanged.
__global__ __launch_bounds__(256) void k_extrapolate(size_t per_loop, int nloops, cd* __restrict__ u,
                                                     const cd* __restrict__ ua, double* __restrict__ T,
                                                     const double* __restrict__ Ta, const double* __restrict__ f) {
    const size_t total = per_loop * (size_t)nloops;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const double c = f[i / per_loop];
        if (c != 0.0) {
            const cd x = u[i], y = ua[i];
            u[i] = cd{x.x + c * (x.x - y.x), x.y + c * (x.y - y.y)};
        }
    }
    if (blockIdx.x == 0)
        for (int l = threadIdx.x; l < nloops; l += blockDim.x)
            if (f[l] != 0.0) T[l] = T[l] + f[l] * (T[l] - Ta[l]);
}

constexpr uint64_t kWsMagic = 0x4c4f4f504f524254ull;  // "LOOPORBT"

struct WsHeader {
    int status;
    int pad;
    uint64_t magic;
};

__global__ void k_ws_init(WsHeader* h) {
    h->status = 0;
    h->magic = kWsMagic;
}

__global__ void k_ws_clear_status(WsHeader* h) { h->status = 0; }

__global__ void k_copy_status(const WsHeader* h, int* status) { *status = h->status; }

// ============================================================================ batched scheduler
// A batch of loops of uneven shape advances in one persistent launch. Each loop belongs to one
// XCD (the chip's eight accelerator dies, each with its own L2 cache), and each XCD works
// through a fixed, totally ordered list of its loops' items (pass, loop, tile):
//   the A tiles of its loops, then for each step the B, C, D and E tiles of its loops.
// A block reads the XCD it runs on from the XCC_ID hardware register and takes items of that
// XCD's list, in order, from that list's counter. Before an item of loop l runs, its block
// waits until loop l's completion counter shows that every earlier item of loop l is done.
// Pass p of a step needs all of pass p-1, and pass B of the next step needs all of the
// previous pass E (which also wrote the next pass A). An item depends only on items earlier in
// its list, and a block that has taken an item is running. So the earliest unfinished item of
// each list can always proceed, and the launch cannot deadlock. Every wait is still bounded in
// time: if one runs out, the block raises an abort flag that every other wait also checks, the
// status becomes LOOP_EHANG, and all blocks leave.
//
// Hand-over between blocks. Producer and consumer of a loop's tiles run on CUs of the same
// XCD and so share its L2: the producer's stores are in that L2 once the wavefront's store
// counter reaches zero, and the consumer invalidates its CU's L1 before it reads. No L2 is
// written back or invalidated per item (an agent-scope release or acquire would do both, for
// the whole L2, which costs far more than the item's work). Kernel boundaries order the launch
// against the kernels before and after it as usual.
//
// The queue and completion counters live in the work space and are cleared by a small kernel
// queued before every launch (k_batch_reset), so that a launch abandoned after a wait ran out
// leaves nothing behind for the next one.
constexpr int kMaxXcd = 16;
struct WsOff {  // byte offsets of one loop's regions inside the work space
    size_t A, BD, Cb, U, G, partial, J, dJdT, Told;
};

struct BatchLoop {
    Shape sh;    // this loop alone (nloops = 1)
    WsOff off;
    size_t uoff;  // offset of the loop's spectrum in the rfft-layout pool (complex values)
    int nt[5];    // tiles of passes A, B, C, D, E
    int ipl;      // items per step: B + C + D + E tiles
};

struct BatchQueue {
    int next[kMaxXcd];  // next item of each XCD's list to hand out
    int abort;          // raised when a bounded wait runs out
    int pad[3];
};

enum : int { PASS_A = 0, PASS_B = 1, PASS_C = 2, PASS_D = 3, PASS_E = 4 };

__host__ __device__ inline uint32_t item_code(int l, int pass, int tile) {
    return ((uint32_t)l << 16) | ((uint32_t)pass << 13) | (uint32_t)tile;
}

struct BatchArgs {
    const BatchLoop* loops;
    const uint32_t* items;  // per XCD x, from items + xoff[x]: nA[x] prologue items, then the ips[x] of one step
    int nloops, nsteps;
    int xlist[kMaxXcd];  // item list of the XCD with each XCC_ID, or -1 for an id the plan never saw
    int xoff[kMaxXcd], nA[kMaxXcd], ips[kMaxXcd];
    BatchQueue* q;
    int* done;  // [nloops] completion counters
    char* ws;
    int* status;
    double* T;
    double* J_hist;  // [nsteps][nloops] or null
    double dtau;
    int scheme;
    const cd* tw;
    unsigned long long spin_ticks;  // bound of one dependency wait, in ticks of the 100 MHz clock
};

constexpr double kWallClockHz = 1e8;       // wall_clock64() runs at 100 MHz
constexpr double kDefaultWaitLimit = 2.0;  // seconds

__device__ __forceinline__ Work batch_work(const BatchLoop& b, char* ws, int* status) {
    Work w{};
    w.A = reinterpret_cast<cd*>(ws + b.off.A);
    w.BD = reinterpret_cast<cd*>(ws + b.off.BD);
    w.Cb = reinterpret_cast<cd*>(ws + b.off.Cb);
    w.U = reinterpret_cast<cd*>(ws + b.off.U);
    w.G = reinterpret_cast<cd*>(ws + b.off.G);
    w.partial = reinterpret_cast<double*>(ws + b.off.partial);
    w.J = reinterpret_cast<double*>(ws + b.off.J);
    w.dJdT = reinterpret_cast<double*>(ws + b.off.dJdT);
    w.Told = reinterpret_cast<double*>(ws + b.off.Told);
    w.status = status;
    return w;
}

// Wait until *cnt >= target. Returns 1 when the launch is being abandoned: this wait ran out
// (it raises the abort flag), or another one did. Either way the status word says LOOP_EHANG,
// so that an abandoned launch never passes for a complete one.
__device__ int wait_count(int* cnt, int target, BatchQueue* q, int* status, unsigned long long spin_ticks) {
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return 0;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(2);
        if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return 0;
        if (__hip_atomic_load(&q->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            wall_clock64() - t0 > spin_ticks) {
            atomicExch(&q->abort, 1);
            atomicCAS(status, 0, LOOP_EHANG);
            return 1;
        }
    }
}

// The XCD (accelerator die) the calling wavefront runs on: XCC_ID, bits 3:0 of hardware
// register 20 on gfx950.
__device__ __forceinline__ int xcc_id() { return (int)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

// Marks in seen[] the XCC_IDs of the XCDs that run this launch's blocks.
__global__ void k_xcc_probe(int* seen) {
    if (threadIdx.x == 0) seen[xcc_id()] = 1;
}

// Calls f(std::integral_constant<int, S>) for the power of two S == n in [LO, HI]; other n do
// nothing (plans only hold sizes their kernels cover).
template <int LO, int HI, class F>
__device__ __forceinline__ void size_switch(int n, F&& f) {
    if constexpr (LO <= HI) {
        if (n == LO)
            f(std::integral_constant<int, LO>{});
        else
            size_switch<2 * LO, HI>(n, static_cast<F&&>(f));
    }
}

// The twiddle table's address as seen by one pass: an opaque copy, so that the compiler does
// not hoist every pass's twiddle cache out of the step loop and keep them all live at once.
__device__ __forceinline__ const cd* per_pass(const cd* tw) {
    asm volatile("" : "+s"(tw));
    return tw;
}

// One pass body per (pass, size), each compiled as its own function so that register
// allocation is per body rather than over the union of all bodies.
template <int N>
__device__ __noinline__ void bk_A(const Shape& sh, int tile, const Work& w, cd* lds, const cd* tw) {
    col_pass_A<N>(sh, tile, w, lds, tw);
}
template <int M>
__device__ __noinline__ void bk_B(const Shape& sh, int tile, const Work& w, cd* lds, const cd* tw) {
    row_pass_B<M>(sh, tile, w, lds, tw);
}
template <int N>
__device__ __noinline__ void bk_C(const Shape& sh, int tile, const double* T, const Work& w, double dtau,
                                  int scheme, cd* lds, double* red, const cd* tw) {
    col_pass_C<N>(sh, tile, T, w, MODE_STEP, dtau, scheme, lds, red, tw);
}
template <int M>
__device__ __noinline__ void bk_D(const Shape& sh, int tile, const Work& w, double* T, double dtau, double* jh,
                                  cd* lds, const cd* tw) {
    row_pass_D<M>(sh, tile, w, T, MODE_STEP, dtau, jh, nullptr, nullptr, lds, tw);
}
template <int N>
__device__ __noinline__ void bk_E(const Shape& sh, int tile, const Work& w, double dtau, int scheme, int fuseA,
                                  cd* lds, const cd* tw) {
    col_pass_E<N>(sh, tile, w, MODE_STEP, dtau, scheme, fuseA != 0, lds, tw);
}

__global__ __launch_bounds__(kBlock) void k_batch(BatchArgs a) {
    constexpr int RH = 512, CH = 1024;  // transform sizes of the batched passes
    extern __shared__ __align__(16) cd lds[];  // 16-byte aligned: one ds_read_b128 per complex value
    __shared__ double red[2 * kBlock / 64];
    __shared__ int s_item, s_stop;
    // the list of the XCD this block runs on (XCC_ID, bits 3:0 of hardware register 20)
    const int x = a.xlist[xcc_id()];
    if (x < 0) {  // an XCD the plan's probe did not see: leave, and say so
        if (threadIdx.x == 0) {
            atomicExch(&a.q->abort, 1);
            atomicCAS(a.status, 0, LOOP_ENOTSUP);
        }
        return;
    }
    const uint32_t* items = a.items + a.xoff[x];
    const int nA = a.nA[x], ips = a.ips[x];
    const int total = nA + a.nsteps * ips;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&a.q->next[x], 1);
        __syncthreads();
        const int i = s_item;
        if (i >= total) break;
        int s = 0;
        uint32_t code;
        if (i < nA) {
            code = items[i];
        } else {
            s = (i - nA) / ips;
            code = items[nA + (i - nA) % ips];
        }
        const int l = (int)(code >> 16), pass = (int)((code >> 13) & 7), tile = (int)(code & 0x1fff);
        const BatchLoop b = a.loops[l];
        int target = 0;
        if (pass != PASS_A) {
            target = b.nt[PASS_A] + s * b.ipl;
            for (int p = PASS_B; p < pass; ++p) target += b.nt[p];
        }
        if (threadIdx.x == 0) s_stop = wait_count(&a.done[l], target, a.q, a.status, a.spin_ticks);
        __syncthreads();
        if (s_stop) break;
        // The producers ran on this XCD: their results are in its L2. Drop this CU's L1 copies
        // of earlier contents before reading (each wavefront, ahead of its own loads).
        asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
        const Work w = batch_work(b, a.ws, a.status);
        const Shape& sh = b.sh;
        switch (pass) {
            case PASS_A:
                size_switch<8, CH>(sh.N, [&](auto c) { bk_A<decltype(c)::value>(sh, tile, w, lds, a.tw); });
                break;
            case PASS_B:
                size_switch<8, RH>(sh.M, [&](auto c) { bk_B<decltype(c)::value>(sh, tile, w, lds, a.tw); });
                break;
            case PASS_C:
                size_switch<8, CH>(sh.N, [&](auto c) {
                    bk_C<decltype(c)::value>(sh, tile, a.T + l, w, a.dtau, a.scheme, lds, red, a.tw);
                });
                break;
            case PASS_D: {
                double* jh = a.J_hist ? a.J_hist + (size_t)s * a.nloops + l : nullptr;
                size_switch<8, RH>(sh.M, [&](auto c) { bk_D<decltype(c)::value>(sh, tile, w, a.T + l, a.dtau, jh, lds, a.tw); });
                break;
            }
            default:
                size_switch<8, CH>(sh.N, [&](auto c) {
                    bk_E<decltype(c)::value>(sh, tile, w, a.dtau, a.scheme, s + 1 < a.nsteps, lds, a.tw);
                });
                break;
        }
        // Every wave waits until its stores have reached this XCD's L2; after the barrier the
        // counter moves. Consumers run on this XCD too, so nothing is written back.
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(&a.done[l], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Queue and completion counters of the persistent schedule, cleared before every launch (a
// kernel rather than a memset, so that the step can be recorded into a graph and replayed):
// a launch abandoned after a wait ran out leaves them partly counted.
__global__ void k_batch_reset(BatchQueue* q, int* done, int nloops) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMaxXcd) q->next[i] = 0;
    if (i == 0) q->abort = 0;
    for (int l = i; l < nloops; l += gridDim.x * blockDim.x) done[l] = 0;
}

// Launch-per-pass form of the same batched step: one kernel per pass covers the tiles of
// every loop (block -> item code), and kernel boundaries order the passes. No counters and
// no fences, at the cost of four launches per step.
//
// Each pass has a few kernel variants, k_rag<PASS, V>. A variant fixes the range of
// transform sizes its size dispatch contains. Registers are allocated for the largest body
// a kernel holds, so a kernel limited to short transforms can keep more wavefronts per SIMD.
// For the row passes a variant also fixes how a tile of rows reaches LDS: staged through
// vector registers (load_rows) or copied by the load unit (load_rows_lds). Every variant
// runs the same arithmetic; a plan starts with the narrowest staged variant that covers its
// sizes, and loop_batch_autotune times the others.
struct RagVariant {
    int lo, hi;  // transform sizes compiled in: powers of two in [lo, hi]
    bool dma;    // row tiles copied straight into LDS
    int pt;      // points per thread of the row transforms (0: the default, 8)
};
constexpr int kRowVariants = 4, kColVariants = 3, kRagVariants = 4;
__host__ __device__ constexpr bool is_row_pass(int pass) { return pass == PASS_B || pass == PASS_D; }
__host__ __device__ constexpr int rag_count(int pass) { return is_row_pass(pass) ? kRowVariants : kColVariants; }
__host__ __device__ constexpr RagVariant rag_variant(int pass, int v) {
    return is_row_pass(pass) ? (v == 0   ? RagVariant{8, 512, false, 0}
                                : v == 1 ? RagVariant{8, 64, false, 0}
                                : v == 2 ? RagVariant{8, 64, true, 0}
                                         : RagVariant{8, 64, false, 4})
                             : (v == 0   ? RagVariant{8, 1024, false, 0}
                                : v == 1 ? RagVariant{8, 64, false, 0}
                                         : RagVariant{8, 512, false, 0});
}
template <int M, int PT>
constexpr int row_pt() {
    return PT ? PT : RowG<M>::PT;
}

template <int PASS, int V>
__global__ __launch_bounds__(kBlock) void k_rag(BatchArgs a, const uint32_t* __restrict__ codes, int s) {
    constexpr RagVariant var = rag_variant(PASS, V);
    extern __shared__ __align__(16) cd lds[];  // 16-byte aligned: one ds_read_b128 per complex value
    __shared__ double red[2 * kBlock / 64];
    const uint32_t code = codes[blockIdx.x];
    const int l = (int)(code >> 16), tile = (int)(code & 0x1fff);
    const BatchLoop b = a.loops[l];
    const Work w = batch_work(b, a.ws, a.status);
    const Shape& sh = b.sh;
    if constexpr (PASS == PASS_A) {
        size_switch<var.lo, var.hi>(sh.N, [&](auto c) { col_pass_A<decltype(c)::value>(sh, tile, w, lds, a.tw); });
    } else if constexpr (PASS == PASS_B) {
        size_switch<var.lo, var.hi>(sh.M, [&](auto c) {
            constexpr int M_ = decltype(c)::value;
            row_pass_B<M_, var.dma, row_pt<M_, var.pt>()>(sh, tile, w, lds, a.tw);
        });
    } else if constexpr (PASS == PASS_C) {
        size_switch<var.lo, var.hi>(sh.N, [&](auto c) {
            col_pass_C<decltype(c)::value>(sh, tile, a.T + l, w, MODE_STEP, a.dtau, a.scheme, lds, red, a.tw);
        });
    } else if constexpr (PASS == PASS_D) {
        double* jh = a.J_hist ? a.J_hist + (size_t)s * a.nloops + l : nullptr;
        size_switch<var.lo, var.hi>(sh.M, [&](auto c) {
            constexpr int M_ = decltype(c)::value;
            row_pass_D<M_, var.dma, row_pt<M_, var.pt>()>(sh, tile, w, a.T + l, MODE_STEP, a.dtau, jh, nullptr,
                                                          nullptr, lds, a.tw);
        });
    } else {
        size_switch<var.lo, var.hi>(sh.N, [&](auto c) {
            col_pass_E<decltype(c)::value>(sh, tile, w, MODE_STEP, a.dtau, a.scheme, s + 1 < a.nsteps, lds, a.tw);
        });
    }
}

// ts: the launch's TraceScope
template <int PASS, class Scope>
void launch_rag(int v, dim3 grid, size_t lds, hipStream_t hs, const BatchArgs& a, const uint32_t* c, int step,
                Scope& ts) {
    const uint32_t sh = (uint32_t)lds;
    switch (v) {
        case 0: ts.launch(k_rag<PASS, 0>, grid, dim3(kBlock), sh, hs, a, c, step); break;
        case 1: ts.launch(k_rag<PASS, 1>, grid, dim3(kBlock), sh, hs, a, c, step); break;
        case 2: ts.launch(k_rag<PASS, 2>, grid, dim3(kBlock), sh, hs, a, c, step); break;
        default:
            if constexpr (is_row_pass(PASS)) ts.launch(k_rag<PASS, 3>, grid, dim3(kBlock), sh, hs, a, c, step);
            break;
    }
}

// LDS-resident step (see resident.hpp): block l runs all nsteps of loop l with its state and
// intermediates in LDS. The rfft-layout spectrum is read at the start and written back at
// the end (the same arithmetic as k_to_band and k_from_band), T[l] likewise.

// LDS-resident step (see resident.hpp): block l runs all nsteps of loop l with its state and
// intermediates in LDS. The rfft-layout spectrum is read at the start and written back at
// the end (the same arithmetic as k_to_band and k_from_band), T[l] likewise.
template <int M, int N>
__global__ __launch_bounds__(kBlock, (ResG<M, N>::BLOCKS_PER_CU)) void k_resident(Shape sh, const cd* uin, cd* uout, double* T, double dtau,
                                                     int scheme, int nsteps, double* J_hist, int* status,
                                                     const cd* __restrict__ tw) {
    using R = ResG<M, N>;
    extern __shared__ __align__(16) cd lds[];  // 16-byte aligned: one ds_read_b128 per complex value
    cd* U = lds;
    cd* A = U + R::S;
    cd* X = A + R::W;
    cd* EX = X + R::W;
    double* part = reinterpret_cast<double*>(EX + R::EX);
    double* sc = part + 2 * R::C;  // T, T_old, J, dJ/dT
    double* red = sc + 4;          // 2 kBlock / 64 doubles
    const int l = blockIdx.x;
    Shape s1 = sh;
    s1.nloops = 1;
    Work w{};
    w.A = A;
    w.BD = X;
    w.Cb = X;
    w.U = U;
    w.G = U;
    w.partial = part;
    w.J = sc + 2;
    w.dJdT = sc + 3;
    w.Told = sc + 1;
    w.status = status;
    const cd* u = uin + (size_t)l * N * sh.H;
    for (int i = threadIdx.x; i < R::S; i += kBlock) {
        const int j = i / R::NB, kk = i % R::NB;
        const int e = (kk <= R::Ks) ? kk : kk + N - R::NB;
        cd v = u[(size_t)e * sh.H + j];
        if (j == 0) {
            const cd pr = u[(size_t)((N - e) & (N - 1)) * sh.H];
            v = cd{0.5 * (v.x + pr.x), 0.5 * (v.y - pr.y)};
        }
        U[i] = v;
    }
    if (threadIdx.x == 0) sc[0] = T[l];
    __syncthreads();
    if (nsteps > 0) {
#pragma unroll 1
        for (int b = 0; b < R::COL_ROUNDS; ++b) col_pass_A<N>(s1, b, w, EX, per_pass(tw));
        __syncthreads();
    }
    for (int st = 0; st < nsteps; ++st) {
#pragma unroll 1
        for (int tile = 0; tile < R::ROW_ROUNDS; ++tile) res_row_B<M>(s1, tile, A, X, EX, per_pass(tw));
        __syncthreads();
#pragma unroll 1
        for (int b = 0; b < R::COL_ROUNDS; ++b)
            col_pass_C<N>(s1, b, sc, w, MODE_STEP, dtau, scheme, EX, red, per_pass(tw));
        __syncthreads();
        // J, dJ/dT and T' from pass C's partials; pass D reads neither T nor the partials
        if (threadIdx.x < 64)
            finalize_loop(s1, 0, w, sc, MODE_STEP, dtau, J_hist ? J_hist + (size_t)st * gridDim.x + l : nullptr,
                          nullptr, nullptr);
#pragma unroll 1
        for (int tile = 0; tile < R::ROW_ROUNDS; ++tile) res_row_D<M>(s1, tile, A, X, EX, per_pass(tw));
        __syncthreads();
#pragma unroll 1
        for (int b = 0; b < R::COL_ROUNDS; ++b)
            col_pass_E<N>(s1, b, w, MODE_STEP, dtau, scheme, st + 1 < nsteps, EX, per_pass(tw));
        __syncthreads();
    }
    cd* o = uout + (size_t)l * N * sh.H;
    for (int i = threadIdx.x; i < N * sh.H; i += kBlock) {
        const int e = i / sh.H, j = i % sh.H;
        const int kk = j < R::C ? band_row(e, N, R::Ks) : -1;
        o[i] = kk >= 0 ? U[j * R::NB + kk] : cd{0.0, 0.0};
    }
    if (threadIdx.x == 0) T[l] = sc[0];
}

// rfft-layout pool -> per-loop band state (blockIdx.z = loop); see k_to_band.
__global__ __launch_bounds__(256) void k_to_band_batch(const BatchLoop* loops, const cd* __restrict__ pool,
                                                       char* ws) {
    __shared__ cd tile[32][33];
    const BatchLoop& b = loops[blockIdx.z];
    const Shape& sh = b.sh;
    const int kk0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    if (kk0 >= sh.NB || j0 >= sh.C) return;
    const int tx = threadIdx.x % 32, ty0 = threadIdx.x / 32;
    const cd* u = pool + b.uoff;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int kk = kk0 + ty, j = j0 + tx;
        cd v{0.0, 0.0};
        if (kk < sh.NB && j < sh.C) {
            const int e = (kk <= sh.Ks) ? kk : kk + sh.N - sh.NB;
            v = u[(size_t)e * sh.H + j];
            if (j == 0) {
                const cd pr = u[(size_t)((sh.N - e) & (sh.N - 1)) * sh.H];
                v = cd{0.5 * (v.x + pr.x), 0.5 * (v.y - pr.y)};
            }
        }
        tile[ty][tx] = v;
    }
    __syncthreads();
    cd* dst = reinterpret_cast<cd*>(ws + b.off.U);
    for (int ty = ty0; ty < 32; ty += 8) {
        const int j = j0 + ty, kk = kk0 + tx;
        if (j < sh.C && kk < sh.NB) dst[(size_t)j * sh.NB + kk] = tile[tx][ty];
    }
}

__global__ __launch_bounds__(256) void k_from_band_batch(const BatchLoop* loops, const char* ws,
                                                         cd* __restrict__ pool) {
    __shared__ cd tile[32][33];
    const BatchLoop& b = loops[blockIdx.z];
    const Shape& sh = b.sh;
    const int e0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    if (e0 >= sh.N || j0 >= sh.H) return;
    const int tx = threadIdx.x % 32, ty0 = threadIdx.x / 32;
    const cd* src = reinterpret_cast<const cd*>(ws + b.off.U);
    for (int ty = ty0; ty < 32; ty += 8) {
        const int j = j0 + ty, e = e0 + tx;
        const int kk = (j < sh.C && e < sh.N) ? band_row(e, sh.N, sh.Ks) : -1;
        tile[ty][tx] = kk >= 0 ? src[(size_t)j * sh.NB + kk] : cd{0.0, 0.0};
    }
    __syncthreads();
    cd* o = pool + b.uoff;
    for (int ty = ty0; ty < 32; ty += 8) {
        const int e = e0 + ty, j = j0 + tx;
        if (e < sh.N && j < sh.H) o[(size_t)e * sh.H + j] = tile[tx][ty];
    }
}

__global__ void k_batch_ws_init(BatchQueue* q, int* done, int nloops) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMaxXcd) q->next[i] = 0;
    if (i == 0) q->abort = 0;
    if (i < nloops) done[i] = 0;
}

// ============================================================================ host side
struct TwTable {
    cd* dev = nullptr;
};

std::mutex g_mu;
std::map<int, TwTable> g_tables;

// exp(-2 pi i t / TW_N) rounded from long double, with exact values on the axes.
void host_twiddles(std::vector<cd>& h) {
    h.resize(TW_N);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int t = 0; t < TW_N; ++t) {
        // reduce to the first octant and rebuild by symmetry so that every entry is as
        // accurate as the long-double evaluation of an angle in [0, pi/4]
        const int q = t / (TW_N / 4), r = t % (TW_N / 4);
        long double c, s;
        if (r == 0) {
            c = 1.0L;
            s = 0.0L;
        } else if (2 * r <= TW_N / 4) {
            const long double a = 2.0L * pi * (long double)r / (long double)TW_N;
            c = cosl(a);
            s = sinl(a);
        } else {
            const long double a = 2.0L * pi * (long double)(TW_N / 4 - r) / (long double)TW_N;
            c = sinl(a);
            s = cosl(a);
        }
        // angle = q * pi/2 + theta with (cos theta, sin theta) = (c, s)
        long double C, S;
        switch (q) {
            case 0: C = c; S = s; break;
            case 1: C = -s; S = c; break;
            case 2: C = -c; S = -s; break;
            default: C = s; S = -c; break;
        }
        h[t] = cd{(double)C, (double)(-S)};  // exp(-i angle)
    }
}

int get_table(const cd** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LOOP_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tables.find(dev);
    if (it != g_tables.end()) {
        *out = it->second.dev;
        return LOOP_OK;
    }
    std::vector<cd> h;
    host_twiddles(h);
    TwTable tb;
    if (hipMalloc((void**)&tb.dev, sizeof(cd) * TW_N) != hipSuccess) return LOOP_EHIP;
    if (hipMemcpy(tb.dev, h.data(), sizeof(cd) * TW_N, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(tb.dev);
        return LOOP_EHIP;
    }
    g_tables[dev] = tb;
    *out = tb.dev;
    return LOOP_OK;
}

// Per device, the address of that device's copy of `scratch` (under g_mu).
std::map<int, char*> g_scratch;

// Record the current device's scratch address. The call allocates nothing; it fails if the
// runtime cannot resolve the symbol on this device.
int init_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LOOP_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch.count(dev)) return LOOP_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return LOOP_EHIP;
    g_scratch[dev] = static_cast<char*>(p);
    return LOOP_OK;
}

// The current device's scratch address and twiddle table, without allocating anything: the
// table must exist already (loop_init, or any earlier call on the device, creates it).
int device_statics(char** base, const cd** tw) {
    int st = init_scratch();
    if (st) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LOOP_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    const auto t = g_tables.find(dev);
    if (t == g_tables.end()) return LOOP_EINVAL;
    *tw = t->second.dev;
    *base = g_scratch[dev];
    return LOOP_OK;
}

bool pow2_in_range(int n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }

int check_shape(double L, int Nx, int Ns, int nloops) {
    if (!(L > 0.0) || !std::isfinite(L)) return LOOP_EINVAL;
    if (nloops < 1 || nloops > 65535) return LOOP_EINVAL;
    if (Nx < 8 || Ns < 8 || Nx > 1024 || Ns > 1024) return LOOP_EINVAL;
    if (!pow2_in_range(Nx) || !pow2_in_range(Ns)) return LOOP_ENOTSUP;
    return LOOP_OK;
}

bool aligned(const void* p, size_t a) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) % a) == 0; }

Shape make_shape(double L, int Nx, int Ns, int nloops) {
    Shape s;
    s.M = Nx;
    s.N = Ns;
    s.Kx = (Nx - 1) / 3;
    s.Ks = (Ns - 1) / 3;
    s.H = Nx / 2 + 1;
    s.C = s.Kx + 1;
    s.NB = 2 * s.Ks + 1;
    s.logN = 0;
    while ((1 << s.logN) < Ns) ++s.logN;
    s.nloops = nloops;
    s.L = L;
    return s;
}

size_t round_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Work space layout: header | A | BD | Cb | U | G | partial | J | dJdT | Told
size_t layout(const Shape& s, char* base, Work* w) {
    size_t off = round_up(sizeof(WsHeader));
    const size_t inter = (size_t)s.nloops * s.N * s.C * sizeof(cd);
    const size_t band = (size_t)s.nloops * s.NB * s.C * sizeof(cd);
    const size_t part = (size_t)s.nloops * s.C * 2 * sizeof(double);
    const size_t scal = (size_t)s.nloops * sizeof(double);
    Work ww{};
    ww.status = reinterpret_cast<int*>(base);
    ww.A = reinterpret_cast<cd*>(base + off); off = round_up(off + inter);
    ww.BD = reinterpret_cast<cd*>(base + off); off = round_up(off + inter);
    ww.Cb = reinterpret_cast<cd*>(base + off); off = round_up(off + inter);
    ww.U = reinterpret_cast<cd*>(base + off); off = round_up(off + band);
    ww.G = reinterpret_cast<cd*>(base + off); off = round_up(off + band);
    ww.partial = reinterpret_cast<double*>(base + off); off = round_up(off + part);
    ww.J = reinterpret_cast<double*>(base + off); off = round_up(off + scal);
    ww.dJdT = reinterpret_cast<double*>(base + off); off = round_up(off + scal);
    ww.Told = reinterpret_cast<double*>(base + off); off = round_up(off + scal);
    if (w) *w = ww;
    return off;
}

int prepare(double L, int Nx, int Ns, int nloops, void* ws, size_t ws_bytes, Shape* sh, Work* w,
            const cd** tw) {
    int st = check_shape(L, Nx, Ns, nloops);
    if (st) return st;
    *sh = make_shape(L, Nx, Ns, nloops);
    if (!aligned(ws, 256)) return LOOP_EINVAL;
    if (layout(*sh, nullptr, nullptr) > ws_bytes) return LOOP_EWORKSPACE;
    layout(*sh, static_cast<char*>(ws), w);
    return get_table(tw);
}

// ---------------------------------------------------------------------------- kernel timing
// While tracing is on (loop_trace_start), each traced launch records two HIP events at its
// kernel's start and end; loop_trace_stop reads them and sums the durations per kernel. Off
// (the default), a TraceScope costs one relaxed atomic load.
std::atomic<int> g_trace_on{0};
struct TraceRec {
    std::string name;
    hipEvent_t a, b;
};
struct TraceStat {
    long long launches = 0;
    double total_us = 0.0, min_us = 1e300, max_us = 0.0;
};
std::mutex g_trace_mu;
std::vector<TraceRec> g_trace_recs;
std::vector<hipEvent_t> g_trace_pool;
std::vector<std::pair<std::string, TraceStat>> g_trace_stats;
bool g_trace_failed = false;

hipEvent_t trace_event() {
    if (!g_trace_pool.empty()) {
        hipEvent_t e = g_trace_pool.back();
        g_trace_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct TraceScope {
    hipEvent_t a = nullptr, b = nullptr;
    bool launched = false;
    std::string name;
    TraceScope(const char* base, int size, hipStream_t s) : TraceScope(base, size, -1, s) {}
    TraceScope(const char* base, int size, int size2, hipStream_t) {
        if (!g_trace_on.load(std::memory_order_relaxed)) return;
        std::lock_guard<std::mutex> g(g_trace_mu);
        a = trace_event();
        b = a ? trace_event() : nullptr;
        if (!a || !b) {
            g_trace_failed = true;
            if (a) g_trace_pool.push_back(a);
            a = b = nullptr;
            return;
        }
        name = std::string(base);
        if (size > 0) name += "<" + std::to_string(size) + (size2 >= 0 ? ", " + std::to_string(size2) : "") + ">";
    }
    // The scope's one launch. While tracing, the dispatch records the start and stop events
    // itself (hipExtLaunchKernelGGL), so the duration is the kernel's own, as a profiler's
    // kernel trace reports it.
    template <class K, class... Args>
    void launch(K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
        if (a) {
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0, args...);
            launched = true;
        } else {
            hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
        }
    }
    ~TraceScope() {
        if (!a) return;
        std::lock_guard<std::mutex> g(g_trace_mu);
        if (!launched) {  // nothing was launched: return the events unused
            g_trace_pool.push_back(a);
            g_trace_pool.push_back(b);
            return;
        }
        g_trace_recs.push_back(TraceRec{name, a, b});
    }
};

// ---------------------------------------------------------------------------- launchers
#define LO_SWITCH_SIZE(n, BODY)                     \
    switch (n) {                                    \
        case 8: { constexpr int S_ = 8; BODY; } break;       \
        case 16: { constexpr int S_ = 16; BODY; } break;     \
        case 32: { constexpr int S_ = 32; BODY; } break;     \
        case 64: { constexpr int S_ = 64; BODY; } break;     \
        case 128: { constexpr int S_ = 128; BODY; } break;   \
        case 256: { constexpr int S_ = 256; BODY; } break;   \
        case 512: { constexpr int S_ = 512; BODY; } break;   \
        case 1024: { constexpr int S_ = 1024; BODY; } break; \
        default: return LOOP_ENOTSUP;                        \
    }

// Calls f(std::integral_constant<int, S>) for the power of two S == n in [LO, HI].
template <int LO, int HI, class F>
void host_size_switch(int n, F&& f) {
    if constexpr (LO <= HI) {
        if (n == LO)
            f(std::integral_constant<int, LO>{});
        else
            host_size_switch<2 * LO, HI>(n, static_cast<F&&>(f));
    }
}

unsigned col_blocks(const Shape& s) {
    const int F = col_per_block(s.N);  // columns per block
    return (unsigned)(((size_t)s.nloops * s.C + F - 1) / F);
}
unsigned row_blocks(const Shape& s) {
    const int rows = 2 * kBlock * (s.M >= 1024 ? 16 : 8) / s.M;
    return (unsigned)(((size_t)s.nloops * s.N + rows - 1) / rows);
}

int launch_A(const Shape& s, const Work& w, const cd* tw, hipStream_t st) {
    LO_SWITCH_SIZE(s.N, TraceScope ts_("k_colA", S_, st);
                   ts_.launch(k_colA<S_>, dim3(col_blocks(s)), dim3(kBlock), 0, st, s, w, tw));
    return LOOP_OK;
}
int launch_B(const Shape& s, const Work& w, const cd* tw, hipStream_t st) {
    LO_SWITCH_SIZE(s.M, TraceScope ts_("k_rowB", S_, st);
                   ts_.launch(k_rowB<S_>, dim3(row_blocks(s)), dim3(kBlock), 0, st, s, w, tw));
    return LOOP_OK;
}
int launch_C(const Shape& s, const double* T, const Work& w, int mode, double dtau, int scheme, const cd* tw,
             hipStream_t st) {
    auto launch = [&](auto md) {
        constexpr int MD = decltype(md)::value;
        LO_SWITCH_SIZE(s.N, TraceScope ts_("k_colC", S_, MD, st);
                       ts_.launch((k_colC<S_, MD>), dim3(col_blocks(s)), dim3(kBlock), 0, st, s, T, w, dtau,
                                          scheme, tw));
        return LOOP_OK;
    };
    switch (mode) {
        case MODE_RESIDUAL: return launch(std::integral_constant<int, MODE_RESIDUAL>{});
        case MODE_COST: return launch(std::integral_constant<int, MODE_COST>{});
        case MODE_GRAD: return launch(std::integral_constant<int, MODE_GRAD>{});
        case MODE_STEP: return launch(std::integral_constant<int, MODE_STEP>{});
        default: return LOOP_EINVAL;
    }
}
int launch_D(const Shape& s, const Work& w, double* T, int mode, double dtau, double* J_hist, double* Jout,
             double* dJdTout, const cd* tw, hipStream_t st) {
    LO_SWITCH_SIZE(s.M, TraceScope ts_("k_rowD", S_, st);
                   ts_.launch(k_rowD<S_>, dim3(row_blocks(s)), dim3(kBlock), 0, st, s, w, T, mode,
                                           dtau, J_hist, Jout, dJdTout, tw));
    return LOOP_OK;
}
int launch_E(const Shape& s, const Work& w, int mode, double dtau, int scheme, int fuseA, const cd* tw,
             hipStream_t st, const double* T = nullptr) {
    auto launch = [&](auto md) {
        constexpr int MD = decltype(md)::value;
        LO_SWITCH_SIZE(s.N, TraceScope ts_("k_colE", S_, MD, st);
                       ts_.launch((k_colE<S_, MD>), dim3(col_blocks(s)), dim3(kBlock), 0, st, s, w, dtau,
                                          scheme, fuseA, tw, T));
        return LOOP_OK;
    };
    switch (mode) {
        case MODE_GRAD: return launch(std::integral_constant<int, MODE_GRAD>{});
        case MODE_STEP: return launch(std::integral_constant<int, MODE_STEP>{});
        case MODE_ADJOINT: return launch(std::integral_constant<int, MODE_ADJOINT>{});
        default: return LOOP_EINVAL;
    }
}
int launch_AC(const Shape& s, const Work& w, const cd* tw, hipStream_t st, bool with_u) {
    if (!with_u) {
        LO_SWITCH_SIZE(s.N, TraceScope ts_("k_colR", S_, st);
                       ts_.launch(k_colR<S_>, dim3(col_blocks(s)), dim3(kBlock), 0, st, s, w, tw));
        return LOOP_OK;
    }
    LO_SWITCH_SIZE(s.N, TraceScope ts_("k_colAC", S_, st);
                   ts_.launch(k_colAC<S_>, dim3(col_blocks(s)), dim3(kBlock), 0, st, s, w, tw));
    return LOOP_OK;
}
void launch_to_band(const Shape& s, const cd* uhat, cd* U, hipStream_t st) {
    dim3 grid((s.NB + 31) / 32, (s.C + 31) / 32, s.nloops);
    TraceScope ts_("k_to_band", 0, st);
    ts_.launch(k_to_band, grid, dim3(256), 0, st, s, uhat, U);
}
void launch_from_band(const Shape& s, const cd* src, cd* out, hipStream_t st) {
    dim3 grid((s.N + 31) / 32, (s.H + 31) / 32, s.nloops);
    TraceScope ts_("k_from_band", 0, st);
    ts_.launch(k_from_band, grid, dim3(256), 0, st, s, src, out);
}

// Raise kernel k's dynamic-LDS limit to `bytes` on the current device, once: the setting is
// host-side state, so later calls (also those recorded into a HIP graph) make no runtime call.
int ensure_lds_limit(const void* k, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LOOP_EHIP;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;
    std::lock_guard<std::mutex> g(mu);
    const auto key = std::make_pair(k, dev);
    const auto it = done.find(key);
    if (it != done.end() && it->second >= bytes) return LOOP_OK;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return LOOP_EHIP;
    done[key] = bytes;
    return LOOP_OK;
}

// ---------------------------------------------------------------------------- expanded form
// The row pass keeps two input tiles and the exchange regions apart in LDS (up to 83 KB),
// so it takes dynamic LDS; rows of up to 512 points.
int launch_xB(const Shape& s, const Work& w, const double* T, const cd* tw, hipStream_t st) {
    int rc = LOOP_ENOTSUP;
    host_size_switch<8, 512>(s.M, [&](auto c) {
        constexpr int M = decltype(c)::value;
        constexpr size_t bytes = XRowG<M>::LDS * sizeof(cd);
        auto k = k_xB<M>;
        if ((rc = ensure_lds_limit(reinterpret_cast<const void*>(k), bytes))) return;
        hipLaunchKernelGGL(k, dim3(row_blocks(s)), dim3(kBlock), bytes, st, s, w, T, tw);
        rc = LOOP_OK;
    });
    return rc;
}

int launch_x_grad_or_step(const Shape& s, const Work& w, double* T, int mode, double dtau, int scheme, int nsteps,
                          double* J_hist, double* Jout, double* dJdTout, const cd* tw, hipStream_t hs) {
    const dim3 cb(col_blocks(s)), th(kBlock);
    int st;
    LO_SWITCH_SIZE(s.N, hipLaunchKernelGGL(k_xA<S_>, cb, th, 0, hs, s, w, tw));
    const int n = mode == MODE_STEP ? nsteps : 1;
    for (int i = 0; i < n; ++i) {
        if ((st = launch_xB(s, w, T, tw, hs))) return st;
        double* jh = (mode == MODE_STEP && J_hist) ? J_hist + (size_t)i * s.nloops : nullptr;
        hipLaunchKernelGGL(k_x_finalize, dim3(s.nloops), dim3(64), 0, hs, s, w, T, mode == MODE_STEP ? MODE_STEP : MODE_COST,
                           dtau, jh, Jout, dJdTout);
        const double* Tl = mode == MODE_STEP ? w.Told : T;
        const int fuse = (mode == MODE_STEP && i + 1 < n) ? 1 : 0;
        LO_SWITCH_SIZE(s.N, hipLaunchKernelGGL(k_xC<S_>, cb, th, 0, hs, s, w, Tl, mode, dtau, scheme, fuse, tw));
    }
    return LOOP_OK;
}

// ---------------------------------------------------------------------------- centre-symmetric form
size_t xi_layout(const Shape& s, char* base, XiWork* w) {
    size_t off = round_up(sizeof(WsHeader));
    const size_t band = (size_t)s.nloops * s.Kx * (s.Ks + 1) * sizeof(cd);
    const size_t inter = (size_t)s.nloops * s.Kx * s.N * sizeof(double);
    const size_t part = (size_t)s.nloops * s.Kx * 2 * sizeof(double);
    const size_t scal = (size_t)s.nloops * sizeof(double);
    XiWork ww{};
    ww.status = reinterpret_cast<int*>(base);
    ww.U = reinterpret_cast<cd*>(base + off); off = round_up(off + band);
    ww.G = reinterpret_cast<cd*>(base + off); off = round_up(off + band);
    ww.A = reinterpret_cast<double*>(base + off); off = round_up(off + inter);
    ww.BD = reinterpret_cast<double*>(base + off); off = round_up(off + inter);
    ww.Cb = reinterpret_cast<double*>(base + off); off = round_up(off + inter);
    ww.partial = reinterpret_cast<double*>(base + off); off = round_up(off + part);
    ww.J = reinterpret_cast<double*>(base + off); off = round_up(off + scal);
    ww.dJdT = reinterpret_cast<double*>(base + off); off = round_up(off + scal);
    ww.Told = reinterpret_cast<double*>(base + off); off = round_up(off + scal);
    if (w) *w = ww;
    return off;
}

unsigned xi_col_blocks(const Shape& s) {
    const int F = col_per_block(s.N);  // column pairs per block
    return (unsigned)(((size_t)s.nloops * ((s.Kx + 1) / 2) + F - 1) / F);
}

int launch_xi_step(const Shape& s, const XiWork& w, double* T, double dtau, int scheme, int nsteps, double* J_hist,
                   const cd* tw, hipStream_t hs) {
    const dim3 cb(xi_col_blocks(s)), rb(row_blocks(s)), th(kBlock);
    if (nsteps > 0) LO_SWITCH_SIZE(s.N, hipLaunchKernelGGL(k_xi_colA<S_>, cb, th, 0, hs, s, w, tw));
    for (int i = 0; i < nsteps; ++i) {
        double* jh = J_hist ? J_hist + (size_t)i * s.nloops : nullptr;
        LO_SWITCH_SIZE(s.M, hipLaunchKernelGGL(k_xi_rowB<S_>, rb, th, 0, hs, s, w, tw));
        LO_SWITCH_SIZE(s.N, hipLaunchKernelGGL(k_xi_colC<S_>, cb, th, 0, hs, s, T, w, dtau, scheme, tw));
        LO_SWITCH_SIZE(s.M, hipLaunchKernelGGL(k_xi_rowD<S_>, rb, th, 0, hs, s, w, T, dtau, jh, tw));
        LO_SWITCH_SIZE(s.N, hipLaunchKernelGGL(k_xi_colE<S_>, cb, th, 0, hs, s, w, dtau, scheme, i + 1 < nsteps ? 1 : 0,
                                               tw));
    }
    return LOOP_OK;
}

// ---------------------------------------------------------------------------- resident form
int last_error() { return hipGetLastError() == hipSuccess ? LOOP_OK : LOOP_EHIP; }

// loop_set_resident: 0 never, 1 where measured faster (default), 2 wherever it fits
std::atomic<int> g_resident{1};

int max_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return v;
}

// LDS bytes of the resident step for this shape, or 0 where it has no kernel.
size_t resident_bytes(int Nx, int Ns) {
    size_t b = 0;
    host_size_switch<8, 128>(Nx, [&](auto m) {
        host_size_switch<8, 512>(Ns, [&](auto n) {
            using R = ResG<decltype(m)::value, decltype(n)::value>;
            if constexpr (R::FITS) b = R::BYTES;
        });
    });
    return b;
}

bool resident_usable(int Nx, int Ns) {
    const size_t b = resident_bytes(Nx, Ns);
    return b > 0 && b <= (size_t)max_lds_per_block();
}

// Whether one resident block covers a pass of this shape in a single round of transforms.
bool resident_one_round(int Nx, int Ns) {
    bool one = false;
    host_size_switch<8, 128>(Nx, [&](auto m) {
        host_size_switch<8, 512>(Ns, [&](auto n) {
            using R = ResG<decltype(m)::value, decltype(n)::value>;
            if constexpr (R::FITS) one = R::COL_ROUNDS == 1 && R::ROW_ROUNDS == 1;
        });
    });
    return one;
}

// The automatic choice, from measurements on MI355X (one 4-wavefront block per loop is
// latency-bound; the per-pass form spreads a pass over more CUs but pays HBM round trips):
// resident wins while every loop gets a CU of its own (nloops up to the CU count), except a
// lone loop or a few loops whose passes need two rounds per block (32 x 256, 64 x 128).
int resident_blocks_per_cu(int Nx, int Ns) {
    int b = 1;
    host_size_switch<8, 128>(Nx, [&](auto m) {
        host_size_switch<8, 512>(Ns, [&](auto n) {
            using R = ResG<decltype(m)::value, decltype(n)::value>;
            if constexpr (R::FITS) b = R::BLOCKS_PER_CU;
        });
    });
    return b;
}

bool resident_preferred(int Nx, int Ns, int nloops) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return false;
    cus *= resident_blocks_per_cu(Nx, Ns);  // resident blocks the chip holds at once
    // Loops beyond the blocks the chip holds at once take further rounds of the resident
    // launch. Measured against the per-pass form, one-round shapes (32 x 32, 64 x 64) stay
    // ahead for two rounds of loops, two-round shapes only within one round and with at least
    // 16 loops.
    const int rounds = (nloops + cus - 1) / cus;
    if (resident_one_round(Nx, Ns)) return rounds <= 2;
    return rounds == 1 && nloops >= 16;
}

int launch_resident(const Shape& s, cd* u, double* T, double dtau, int scheme, int nsteps, double* J_hist,
                    int* status, const cd* tw, hipStream_t hs) {
    int st = LOOP_ENOTSUP;
    host_size_switch<8, 128>(s.M, [&](auto m) {
        host_size_switch<8, 512>(s.N, [&](auto n) {
            constexpr int M_ = decltype(m)::value, N_ = decltype(n)::value;
            using R = ResG<M_, N_>;
            if constexpr (R::FITS) {
                auto k = k_resident<M_, N_>;
                if ((st = ensure_lds_limit(reinterpret_cast<const void*>(k), R::BYTES))) return;
                TraceScope ts_("k_resident", M_, N_, hs);
                ts_.launch(k, dim3(s.nloops), dim3(kBlock), R::BYTES, hs, s, u, u, T, dtau, scheme, nsteps,
                                   J_hist, status, tw);
                st = last_error();
            }
        });
    });
    return st;
}

// ---------------------------------------------------------------------------- batch plans
struct BatchPlan {
    int device = -1;
    int nloops = 0;
    std::vector<BatchLoop> loops;
    BatchLoop* d_loops = nullptr;
    uint32_t* d_items = nullptr;
    int nxcd = 1;                   // XCDs of the device: one item list each (persistent schedule)
    int xlist[kMaxXcd] = {};        // item list of each XCC_ID, -1 for ids not seen
    int xoff[kMaxXcd] = {}, nA[kMaxXcd] = {}, ips[kMaxXcd] = {};
    size_t ws_bytes = 0, q_off = 0, done_off = 0, pool_elems = 0;
    int max_nb = 1, max_c = 1, max_n = 1, max_h = 1;
    size_t lds_bytes = 0;
    int grid = 1;
    uint32_t* d_pass_codes = nullptr;  // all loops' tiles, pass by pass (A, B, C, D, E)
    int pass_off[6] = {0, 0, 0, 0, 0, 0};
    int schedule = 0;                  // LOOP_BATCH_PER_PASS, LOOP_BATCH_PERSISTENT or LOOP_BATCH_STREAMS
    double wait_limit = kDefaultWaitLimit;  // seconds: bound of one dependency wait (persistent)
    int variant[5] = {0, 0, 0, 0, 0};  // k_rag variant of each pass
    size_t pass_lds[5][kRagVariants] = {};  // dynamic LDS of each pass's launches, per variant
    int min_m = 1 << 30, max_m = 0, min_n = 1 << 30, max_n2 = 0;  // transform sizes present
    // multi-stream schedule: for K = 2, 3, 4 groups of about equal work, the tiles of each
    // group and pass; group g > 0 runs on the plan's stream sx[g - 1] (default priority)
    int nstreams = 2;
    uint32_t* d_group_codes = nullptr;
    int group_off[3][4][6] = {};  // [K - 2][group][pass .. pass + 1]
    hipStream_t sx[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_lag[3] = {nullptr, nullptr, nullptr}, ev_join[3] = {nullptr, nullptr, nullptr};
};

int col_tiles(const Shape& s) { return (s.C + col_per_block(s.N) - 1) / col_per_block(s.N); }
int row_tiles(const Shape& s) {
    const int rows = 4096 / s.M;
    return (s.N + rows - 1) / rows;
}
size_t pass_lds_bytes(const Shape& s) {
    const size_t col = (size_t)col_per_block(s.N) * (s.N + s.N / 8);  // F columns of N + N/8 values
    const int rows = 4096 / s.M, cmax = (s.M - 1) / 3 + 1;
    // two input tiles, or the exchange regions: kBlock / (M/8) pairs of 9M/8 values (rows <= 512)
    const size_t row = std::max<size_t>(2 * (size_t)cmax * (rows + 1), (size_t)kBlock * 9);
    return std::max(col, row) * sizeof(cd);
}
// Dynamic LDS of one pass of the launch-per-pass form for a loop of this shape (row passes:
// with 8 or 4 points per thread).
size_t rag_lds_bytes(const Shape& s, int pass, int pt) {
    size_t n = 0;
    auto row = [&](auto c) {
        constexpr int M_ = decltype(c)::value;
        if constexpr (M_ <= 64) {
            if (pt == 4) {
                using G = RowG<M_, 4>;
                n = pass == PASS_B ? G::LDS_B : G::LDS;
                return;
            }
        }
        using G = RowG<M_>;
        n = pass == PASS_B ? G::LDS_B : G::LDS;
    };
    auto col = [&](auto c) { n = ColG<decltype(c)::value>::LDS; };
    if (is_row_pass(pass))
        host_size_switch<8, 512>(s.M, row);
    else
        host_size_switch<8, 1024>(s.N, col);
    return n * sizeof(cd);
}
bool rag_covers(const BatchPlan* p, int pass, int v) {
    if (v < 0 || v >= rag_count(pass)) return false;
    const RagVariant r = rag_variant(pass, v);
    const int lo = is_row_pass(pass) ? p->min_m : p->min_n, hi = is_row_pass(pass) ? p->max_m : p->max_n2;
    return r.lo <= lo && hi <= r.hi;
}
// The narrowest staged variant covering the plan's sizes.
int rag_default(const BatchPlan* p, int pass) {
    int best = 0;
    for (int v = 0; v < rag_count(pass); ++v) {
        const RagVariant r = rag_variant(pass, v), b = rag_variant(pass, best);
        if (!r.dma && !r.pt && rag_covers(p, pass, v) && r.hi - r.lo < b.hi - b.lo) best = v;
    }
    return best;
}

void free_plan(BatchPlan* p) {
    if (!p) return;
    int dev0 = 0;
    hipGetDevice(&dev0);
    if (p->device >= 0) hipSetDevice(p->device);
    if (p->d_loops) hipFree(p->d_loops);
    if (p->d_items) hipFree(p->d_items);
    if (p->d_pass_codes) hipFree(p->d_pass_codes);
    if (p->d_group_codes) hipFree(p->d_group_codes);
    if (p->ev_fork) hipEventDestroy(p->ev_fork);
    for (int k = 0; k < 3; ++k) {
        if (p->ev_lag[k]) hipEventDestroy(p->ev_lag[k]);
        if (p->ev_join[k]) hipEventDestroy(p->ev_join[k]);
        if (p->sx[k]) hipStreamDestroy(p->sx[k]);
    }
    hipSetDevice(dev0);
    delete p;
}

unsigned elem_blocks(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b ? b : 1);
}


}  // namespace

namespace {
// Argument checks shared by loop_step and loop_step_noalloc.
int step_args(const double* T, const double* uhat, double dtau, int scheme, int nsteps, const double* J_hist) {
    if (!aligned(T, 8) || !aligned(uhat, 16) || (J_hist && !aligned(J_hist, 8))) return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1) || nsteps < 0) return LOOP_EINVAL;
    return LOOP_OK;
}

// The steps of loop_step on a prepared work space: the resident form, or the per-pass kernels
// between the conversions into and out of the band layout.
int step_impl(const Shape& s, const Work& w, const cd* tw, double* T, cd* u, double dtau, int scheme, int nsteps,
              double* J_hist, hipStream_t hs) {
    int st;
    if (loop_step_form(s.M, s.N, s.nloops) == 1)
        return launch_resident(s, u, T, dtau, scheme, nsteps, J_hist, w.status, tw, hs);
    launch_to_band(s, u, w.U, hs);
    if (nsteps > 0 && (st = launch_A(s, w, tw, hs))) return st;
    for (int i = 0; i < nsteps; ++i) {
        double* jh = J_hist ? J_hist + (size_t)i * s.nloops : nullptr;
        if ((st = launch_B(s, w, tw, hs))) return st;
        if ((st = launch_C(s, T, w, MODE_STEP, dtau, scheme, tw, hs))) return st;
        if ((st = launch_D(s, w, T, MODE_STEP, dtau, jh, nullptr, nullptr, tw, hs))) return st;
        if ((st = launch_E(s, w, MODE_STEP, dtau, scheme, i + 1 < nsteps, tw, hs))) return st;
    }
    launch_from_band(s, w.U, u, hs);
    return last_error();
}
}  // namespace

// ============================================================================ C ABI
// Configurations chosen by loop_batch_autotune, per device and multiset of (Nx, Ns), for
// the plans created later in the process.
struct TunedConfig {
    int schedule, nstreams;
    int variant[5];
};
std::mutex g_tune_mu;
std::map<std::vector<int>, TunedConfig>& tune_cache() {
    static std::map<std::vector<int>, TunedConfig> m;
    return m;
}
std::vector<int> plan_signature(const BatchPlan* p) {
    std::vector<std::pair<int, int>> sh;
    for (const BatchLoop& b : p->loops) sh.emplace_back(b.sh.M, b.sh.N);
    std::sort(sh.begin(), sh.end());
    std::vector<int> key{p->device};
    for (const auto& x : sh) {
        key.push_back(x.first);
        key.push_back(x.second);
    }
    return key;
}

extern "C" {

int loop_init(void) {
    const cd* tw = nullptr;
    const int st = get_table(&tw);
    return st ? st : init_scratch();
}

int loop_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev0 = 0;
    hipGetDevice(&dev0);
    for (auto& kv : g_tables) {
        hipSetDevice(kv.first);
        hipFree(kv.second.dev);
    }
    hipSetDevice(dev0);
    g_tables.clear();
    return LOOP_OK;
}

int loop_workspace_bytes(int Nx, int Ns, int nloops, size_t* bytes) {
    if (!bytes) return LOOP_EINVAL;
    int st = check_shape(1.0, Nx, Ns, nloops);
    if (st) return st;
    *bytes = layout(make_shape(1.0, Nx, Ns, nloops), nullptr, nullptr);
    return LOOP_OK;
}

int loop_workspace_init(void* ws, size_t ws_bytes, void* stream) {
    if (!aligned(ws, 256) || ws_bytes < sizeof(WsHeader)) return LOOP_EINVAL;
    hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(1), 0, (hipStream_t)stream, (WsHeader*)ws);
    return last_error();
}

int loop_residual(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat, double* rhat,
                  void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(rhat, 16) || (const void*)uhat == (const void*)rhat)
        return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    launch_to_band(s, reinterpret_cast<const cd*>(uhat), w.U, hs);
    if ((st = launch_A(s, w, tw, hs))) return st;
    if ((st = launch_B(s, w, tw, hs))) return st;
    if ((st = launch_C(s, T, w, MODE_RESIDUAL, 0.0, 0, tw, hs))) return st;
    launch_from_band(s, w.G, reinterpret_cast<cd*>(rhat), hs);
    return last_error();
}

int loop_cost(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat, double* J, void* ws,
              size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(J, 8)) return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    launch_to_band(s, reinterpret_cast<const cd*>(uhat), w.U, hs);
    if ((st = launch_A(s, w, tw, hs))) return st;
    if ((st = launch_B(s, w, tw, hs))) return st;
    if ((st = launch_C(s, T, w, MODE_COST, 0.0, 0, tw, hs))) return st;
    hipLaunchKernelGGL(k_finalize, dim3(nloops), dim3(64), 0, hs, s, w, const_cast<double*>(T), J,
                       (double*)nullptr);
    return last_error();
}

int loop_adjoint_grad(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat, double* Ghat,
                      double* dJdT, double* J, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(Ghat, 16) || (const void*)uhat == (const void*)Ghat)
        return LOOP_EINVAL;
    if ((dJdT && !aligned(dJdT, 8)) || (J && !aligned(J, 8))) return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    launch_to_band(s, reinterpret_cast<const cd*>(uhat), w.U, hs);
    if ((st = launch_A(s, w, tw, hs))) return st;
    if ((st = launch_B(s, w, tw, hs))) return st;
    if ((st = launch_C(s, T, w, MODE_GRAD, 0.0, 0, tw, hs))) return st;
    if ((st = launch_D(s, w, const_cast<double*>(T), MODE_GRAD, 0.0, nullptr, J, dJdT, tw, hs))) return st;
    if ((st = launch_E(s, w, MODE_GRAD, 0.0, 0, 0, tw, hs))) return st;
    launch_from_band(s, w.G, reinterpret_cast<cd*>(Ghat), hs);
    return last_error();
}

int loop_cost_grad(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat, const double* gJ,
                   double* grad_uhat, double* grad_T, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(grad_uhat, 16) || !aligned(grad_T, 8) ||
        (gJ && !aligned(gJ, 8)) || (const void*)uhat == (const void*)grad_uhat)
        return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    launch_to_band(s, reinterpret_cast<const cd*>(uhat), w.U, hs);
    if ((st = launch_A(s, w, tw, hs))) return st;
    if ((st = launch_B(s, w, tw, hs))) return st;
    if ((st = launch_C(s, T, w, MODE_GRAD, 0.0, 0, tw, hs))) return st;
    if ((st = launch_D(s, w, const_cast<double*>(T), MODE_GRAD, 0.0, nullptr, nullptr, nullptr, tw, hs))) return st;
    if ((st = launch_E(s, w, MODE_GRAD, 0.0, 0, 0, tw, hs))) return st;
    dim3 grid((s.N + 31) / 32, (s.H + 31) / 32, s.nloops);
    hipLaunchKernelGGL(k_grad_from_band, grid, dim3(256), 0, hs, s, w.G, gJ, reinterpret_cast<cd*>(grad_uhat));
    hipLaunchKernelGGL(k_grad_T, dim3((nloops + 255) / 256), dim3(256), 0, hs, nloops, gJ, w.dJdT, grad_T);
    return last_error();
}

int loop_to_band(int Nx, int Ns, int nloops, const double* uhat, double* uband, void* stream) {
    int st = check_shape(1.0, Nx, Ns, nloops);
    if (st) return st;
    if (!aligned(uhat, 16) || !aligned(uband, 16) || (const void*)uhat == (const void*)uband) return LOOP_EINVAL;
    launch_to_band(make_shape(1.0, Nx, Ns, nloops), reinterpret_cast<const cd*>(uhat), reinterpret_cast<cd*>(uband),
                   (hipStream_t)stream);
    return last_error();
}

int loop_from_band(int Nx, int Ns, int nloops, const double* uband, double* uhat, void* stream) {
    int st = check_shape(1.0, Nx, Ns, nloops);
    if (st) return st;
    if (!aligned(uhat, 16) || !aligned(uband, 16) || (const void*)uhat == (const void*)uband) return LOOP_EINVAL;
    launch_from_band(make_shape(1.0, Nx, Ns, nloops), reinterpret_cast<const cd*>(uband), reinterpret_cast<cd*>(uhat),
                     (hipStream_t)stream);
    return last_error();
}

namespace {
// The field state of a reverse-mode call: rfft layout converted into the work space's band
// array (canonical), or a caller-owned band array read in place (column 0 through its
// Hermitian part).
int bind_state(const Shape& s, Work& w, int layout, const double* u, hipStream_t hs) {
    if (layout == LOOP_LAYOUT_RFFT) {
        launch_to_band(s, reinterpret_cast<const cd*>(u), w.U, hs);
        w.herm0 = 0;
    } else if (layout == LOOP_LAYOUT_BAND) {
        w.U = const_cast<cd*>(reinterpret_cast<const cd*>(u));
        w.herm0 = 1;
    } else {
        return LOOP_EINVAL;
    }
    return LOOP_OK;
}
}  // namespace

int loop_cost_fwd(double L, int Nx, int Ns, int nloops, int layout, const double* T, const double* u, double* J,
                  double* dJdT, double* rsave, double* usave, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w;
    const cd* tw;
    if (layout != LOOP_LAYOUT_RFFT && layout != LOOP_LAYOUT_BAND) return LOOP_EINVAL;
    if (!aligned(T, 8) || !aligned(u, 16) || !aligned(J, 8) || !aligned(rsave, 16) || (dJdT && !aligned(dJdT, 8)) ||
        (const void*)u == (const void*)rsave || (usave && (!aligned(usave, 16) || usave == rsave || usave == u)))
        return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    if ((st = bind_state(s, w, layout, u, hs))) return st;
    w.G = reinterpret_cast<cd*>(rsave);  // pass C writes the residual there
    if (usave) w.A = reinterpret_cast<cd*>(usave);  // pass A leaves u on the s grid there
    if ((st = launch_A(s, w, tw, hs))) return st;
    if ((st = launch_B(s, w, tw, hs))) return st;
    if ((st = launch_C(s, T, w, MODE_RESIDUAL, 0.0, 0, tw, hs))) return st;
    {
        TraceScope ts_("k_finalize", 0, hs);
        ts_.launch(k_finalize, dim3(nloops), dim3(64), 0, hs, s, w, const_cast<double*>(T), J, dJdT);
    }
    return last_error();
}

int loop_cost_bwd(double L, int Nx, int Ns, int nloops, int layout, const double* T, const double* u,
                  const double* rsave, const double* usave, const double* dJdT, const double* gJ, double* grad_u,
                  double* grad_T, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w;
    const cd* tw;
    if (layout != LOOP_LAYOUT_RFFT && layout != LOOP_LAYOUT_BAND) return LOOP_EINVAL;
    if (!aligned(T, 8) || !aligned(u, 16) || !aligned(rsave, 16) || !aligned(grad_u, 16) || (gJ && !aligned(gJ, 8)) ||
        (const void*)grad_u == (const void*)u || (const void*)grad_u == (const void*)rsave ||
        (usave && (!aligned(usave, 16) || (const void*)grad_u == (const void*)usave)))
        return LOOP_EINVAL;
    if (grad_T && (!aligned(grad_T, 8) || !aligned(dJdT, 8))) return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    // the spectrum itself is read only to recompute u on the s grid
    if (!usave && (st = bind_state(s, w, layout, u, hs))) return st;
    w.R = reinterpret_cast<const cd*>(rsave);
    w.gJ = gJ;
    w.dJdT_in = dJdT;
    w.grad_T = grad_T;  // pass E writes gJ dJ/dT
    cd* gout = w.G;  // band result in the work space, converted below (rfft layout)
    if (layout == LOOP_LAYOUT_BAND) w.G = reinterpret_cast<cd*>(grad_u);
    if (usave) w.A = const_cast<cd*>(reinterpret_cast<const cd*>(usave));  // u on the s grid, from the forward
    if ((st = launch_AC(s, w, tw, hs, usave == nullptr))) return st;
    if ((st = launch_D(s, w, const_cast<double*>(T), MODE_ADJOINT, 0.0, nullptr, nullptr, nullptr, tw, hs))) return st;
    if ((st = launch_E(s, w, MODE_ADJOINT, 0.0, 0, 0, tw, hs, T))) return st;
    if (layout == LOOP_LAYOUT_RFFT) launch_from_band(s, gout, reinterpret_cast<cd*>(grad_u), hs);
    return last_error();
}

int loop_update_grad(double L, int Nx, int Ns, int nloops, int layout, double* T, double* u, const double* grad_u,
                     const double* grad_T, double dtau, int scheme, void* stream) {
    int st = check_shape(L, Nx, Ns, nloops);
    if (st) return st;
    if (layout != LOOP_LAYOUT_RFFT && layout != LOOP_LAYOUT_BAND) return LOOP_EINVAL;
    if (!aligned(T, 8) || !aligned(u, 16) || !aligned(grad_u, 16) || !aligned(grad_T, 8) ||
        (const void*)u == (const void*)grad_u)
        return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1)) return LOOP_EINVAL;
    const Shape s = make_shape(L, Nx, Ns, nloops);
    hipStream_t hs = (hipStream_t)stream;
    if (layout == LOOP_LAYOUT_RFFT) {
        TraceScope ts_("k_update_grad", 0, hs);
        ts_.launch(k_update_grad, dim3(elem_blocks((size_t)s.nloops * s.N * s.H)), dim3(256), 0, hs, s, T,
                           reinterpret_cast<cd*>(u), reinterpret_cast<const cd*>(grad_u), dtau, scheme);
    } else {
        TraceScope ts_("k_update_grad_band", 0, hs);
        ts_.launch(k_update_grad_band, dim3(elem_blocks((size_t)s.nloops * s.C * s.NB)), dim3(256), 0, hs, s,
                           T, reinterpret_cast<cd*>(u), reinterpret_cast<const cd*>(grad_u), dtau, scheme);
    }
    {
        TraceScope ts_("k_update_T", 0, hs);
        ts_.launch(k_update_T, dim3((nloops + 255) / 256), dim3(256), 0, hs, nloops, T, grad_T, dtau);
    }
    return last_error();
}

int loop_step(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme, int nsteps,
              double* J_hist, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    int st = step_args(T, uhat, dtau, scheme, nsteps, J_hist);
    if (st) return st;
    if ((st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw))) return st;
    return step_impl(s, w, tw, T, reinterpret_cast<cd*>(uhat), dtau, scheme, nsteps, J_hist, (hipStream_t)stream);
}

int loop_step_noalloc(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                      int nsteps, double* J_hist, int* status, void* stream) {
    int st = step_args(T, uhat, dtau, scheme, nsteps, J_hist);
    if (st) return st;
    if (status && !aligned(status, 4)) return LOOP_EINVAL;
    if ((st = check_shape(L, Nx, Ns, nloops))) return st;
    const Shape s = make_shape(L, Nx, Ns, nloops);
    if (layout(s, nullptr, nullptr) > kScratchBytes) return LOOP_EWORKSPACE;
    // the device's scratch address and twiddle table, both set up by loop_init: nothing here allocates
    char* base = nullptr;
    const cd* tw = nullptr;
    if ((st = device_statics(&base, &tw))) return st;
    Work w{};
    layout(s, base, &w);
    hipStream_t hs = (hipStream_t)stream;
    // the previous call's status word is cleared by a kernel (not a memset, so that the call can
    // be recorded into a HIP graph and replayed)
    hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(1), 0, hs, reinterpret_cast<WsHeader*>(base));
    if ((st = step_impl(s, w, tw, T, reinterpret_cast<cd*>(uhat), dtau, scheme, nsteps, J_hist, hs))) return st;
    if (status) hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, hs, reinterpret_cast<const WsHeader*>(base), status);
    return last_error();
}

int loop_expanded_grad(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat, double* Ghat,
                       double* dJdT, double* J, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(Ghat, 16) || (const void*)uhat == (const void*)Ghat)
        return LOOP_EINVAL;
    if ((dJdT && !aligned(dJdT, 8)) || (J && !aligned(J, 8))) return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    if (Nx > 512 || (size_t)s.C * s.NB < (size_t)s.N) return LOOP_ENOTSUP;
    hipStream_t hs = (hipStream_t)stream;
    launch_to_band(s, reinterpret_cast<const cd*>(uhat), w.U, hs);
    if ((st = launch_x_grad_or_step(s, w, const_cast<double*>(T), MODE_GRAD, 0.0, 0, 1, nullptr, J, dJdT, tw, hs)))
        return st;
    launch_from_band(s, w.G, reinterpret_cast<cd*>(Ghat), hs);
    return last_error();
}

int loop_step_expanded(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                       int nsteps, double* J_hist, void* ws, size_t ws_bytes, void* stream) {
    Shape s;
    Work w{};
    const cd* tw;
    if (!aligned(T, 8) || !aligned(uhat, 16) || (J_hist && !aligned(J_hist, 8))) return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1) || nsteps < 0) return LOOP_EINVAL;
    int st = prepare(L, Nx, Ns, nloops, ws, ws_bytes, &s, &w, &tw);
    if (st) return st;
    if (Nx > 512 || (size_t)s.C * s.NB < (size_t)s.N) return LOOP_ENOTSUP;
    hipStream_t hs = (hipStream_t)stream;
    cd* u = reinterpret_cast<cd*>(uhat);
    launch_to_band(s, u, w.U, hs);
    if (nsteps > 0 &&
        (st = launch_x_grad_or_step(s, w, T, MODE_STEP, dtau, scheme, nsteps, J_hist, nullptr, nullptr, tw, hs)))
        return st;
    launch_from_band(s, w.U, u, hs);
    return last_error();
}

int loop_extrapolate(int Nx, int Ns, int nloops, double* T, double* uhat, const double* T_a, const double* uhat_a,
                     const double* factor, void* stream) {
    int st = check_shape(22.0, Nx, Ns, nloops);
    if (st) return st;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(T_a, 8) || !aligned(uhat_a, 16) || !aligned(factor, 8))
        return LOOP_EINVAL;
    const size_t per = (size_t)Ns * (Nx / 2 + 1);
    hipLaunchKernelGGL(k_extrapolate, dim3(elem_blocks(per * nloops)), dim3(256), 0, (hipStream_t)stream, per, nloops,
                       reinterpret_cast<cd*>(uhat), reinterpret_cast<const cd*>(uhat_a), T, T_a, factor);
    return last_error();
}

int loop_converge(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                  double J_tol, int stride, long long max_steps, int accelerate, double sqrtJ_first,
                  long long* steps, int* extrapolations, double* J_final, void* ws, size_t ws_bytes, void* stream) {
    int st = check_shape(L, Nx, Ns, nloops);
    if (st) return st;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !steps || !extrapolations || !J_final) return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1) || !(J_tol > 0.0) || stride < 1 ||
        max_steps < 0 || !(sqrtJ_first > 0.0))
        return LOOP_EINVAL;
    hipStream_t hs = (hipStream_t)stream;
    const size_t per = (size_t)Ns * (Nx / 2 + 1), ubytes = sizeof(cd) * per * nloops, tbytes = sizeof(double) * nloops;
    // device buffers: interval anchors (u, T), saved results (u, T), J, extrapolation factors
    char* buf = nullptr;
    const size_t need = 2 * ubytes + 4 * tbytes + 256;
    if (hipMalloc((void**)&buf, need) != hipSuccess) return LOOP_EHIP;
    cd* ua = reinterpret_cast<cd*>(buf);
    cd* ur = reinterpret_cast<cd*>(buf + ubytes);
    double* Ta = reinterpret_cast<double*>(buf + 2 * ubytes);
    double* Tr = Ta + nloops;
    double* dJ = Tr + nloops;
    double* df = dJ + nloops;
    cd* u = reinterpret_cast<cd*>(uhat);
    std::vector<double> J(nloops), Jan(nloops, -1.0), f(nloops, 0.0);
    std::vector<char> done(nloops, 0);
    auto fail = [&](int code) {
        hipFree(buf);
        return code;
    };
    auto cost = [&]() -> int {
        int c = loop_cost(L, Nx, Ns, nloops, T, uhat, dJ, ws, ws_bytes, stream);
        if (c) return c;
        if (hipMemcpyAsync(J.data(), dJ, tbytes, hipMemcpyDeviceToHost, hs) != hipSuccess) return LOOP_EHIP;
        if (hipStreamSynchronize(hs) != hipSuccess) return LOOP_EHIP;
        for (int l = 0; l < nloops; ++l)
            if (!std::isfinite(J[l])) return LOOP_ENONFINITE;
        return LOOP_OK;
    };
    auto copy_loop = [&](cd* dst_u, double* dst_T, const cd* src_u, const double* src_T, int l) -> bool {
        return hipMemcpyAsync(dst_u + per * l, src_u + per * l, sizeof(cd) * per, hipMemcpyDeviceToDevice, hs) ==
                   hipSuccess &&
               hipMemcpyAsync(dst_T + l, src_T + l, sizeof(double), hipMemcpyDeviceToDevice, hs) == hipSuccess;
    };
    auto finish = [&](int l, long long n) -> bool {  // loop l converged at step n: keep its state
        done[l] = 1;
        steps[l] = n;
        J_final[l] = J[l];
        return copy_loop(ur, Tr, u, T, l);
    };
    for (int l = 0; l < nloops; ++l) {
        steps[l] = -1;
        extrapolations[l] = 0;
    }
    // the initial state (loop_step makes it canonical in place, as the steps below would)
    if ((st = loop_step(L, Nx, Ns, nloops, T, uhat, dtau, scheme, 0, nullptr, ws, ws_bytes, stream))) return fail(st);
    if ((st = cost())) return fail(st);
    long long n = 0;
    int left = nloops;
    for (int l = 0; l < nloops; ++l)
        if (J[l] < J_tol) {
            if (!finish(l, 0)) return fail(LOOP_EHIP);
            --left;
        }
    while (left > 0 && n < max_steps) {
        if ((st = loop_step(L, Nx, Ns, nloops, T, uhat, dtau, scheme, stride, nullptr, ws, ws_bytes, stream)))
            return fail(st);
        n += stride;
        if ((st = cost())) return fail(st);
        bool any = false;
        for (int l = 0; l < nloops; ++l) {
            f[l] = 0.0;
            if (done[l]) continue;
            if (J[l] < J_tol) {
                if (!finish(l, n)) return fail(LOOP_EHIP);
                --left;
                continue;
            }
            if (!accelerate) continue;
            if (Jan[l] < 0.0) {
                if (std::sqrt(J[l]) <= sqrtJ_first) {
                    if (!copy_loop(ua, Ta, u, T, l)) return fail(LOOP_EHIP);
                    Jan[l] = J[l];
                }
            } else if (std::sqrt(J[l]) <= 0.5 * std::sqrt(Jan[l])) {
                const double rho = std::sqrt(J[l] / Jan[l]);
                f[l] = rho / (1.0 - rho);
                any = true;
            }
        }
        if (!any) continue;
        if (hipMemcpyAsync(df, f.data(), tbytes, hipMemcpyHostToDevice, hs) != hipSuccess) return fail(LOOP_EHIP);
        if ((st = loop_extrapolate(Nx, Ns, nloops, T, uhat, Ta, reinterpret_cast<const double*>(ua), df, stream)))
            return fail(st);
        if ((st = cost())) return fail(st);
        for (int l = 0; l < nloops; ++l) {
            if (f[l] == 0.0) continue;
            ++extrapolations[l];
            if (J[l] < J_tol) {
                if (!finish(l, n)) return fail(LOOP_EHIP);
                --left;
            } else {
                if (!copy_loop(ua, Ta, u, T, l)) return fail(LOOP_EHIP);
                Jan[l] = J[l];
            }
        }
    }
    // converged loops return the state at which they converged; the others their last state
    for (int l = 0; l < nloops; ++l) {
        if (done[l]) {
            if (!copy_loop(u, T, ur, Tr, l)) return fail(LOOP_EHIP);
        } else {
            J_final[l] = J[l];
        }
    }
    if (hipStreamSynchronize(hs) != hipSuccess) return fail(LOOP_EHIP);
    hipFree(buf);
    return LOOP_OK;
}

int loop_step_xi_workspace_bytes(int Nx, int Ns, int nloops, size_t* bytes) {
    int st = check_shape(22.0, Nx, Ns, nloops);
    if (st) return st;
    if (!bytes) return LOOP_EINVAL;
    *bytes = xi_layout(make_shape(22.0, Nx, Ns, nloops), nullptr, nullptr);
    return LOOP_OK;
}

int loop_step_xi(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme, int nsteps,
                 double* J_hist, void* ws, size_t ws_bytes, void* stream) {
    int st = check_shape(L, Nx, Ns, nloops);
    if (st) return st;
    if (Nx > 512) return LOOP_ENOTSUP;  // row tiles of the real intermediates, as the batched form
    if (!aligned(T, 8) || !aligned(uhat, 16) || (J_hist && !aligned(J_hist, 8)) || !aligned(ws, 256))
        return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1) || nsteps < 0) return LOOP_EINVAL;
    const Shape s = make_shape(L, Nx, Ns, nloops);
    if (xi_layout(s, nullptr, nullptr) > ws_bytes) return LOOP_EWORKSPACE;
    XiWork w;
    xi_layout(s, static_cast<char*>(ws), &w);
    const cd* tw;
    if ((st = get_table(&tw))) return st;
    hipStream_t hs = (hipStream_t)stream;
    cd* u = reinterpret_cast<cd*>(uhat);
    hipLaunchKernelGGL(k_to_xi, dim3(elem_blocks((size_t)nloops * s.Kx * (s.Ks + 1))), dim3(256), 0, hs, s, u, w.U);
    if ((st = launch_xi_step(s, w, T, dtau, scheme, nsteps, J_hist, tw, hs))) return st;
    hipLaunchKernelGGL(k_from_xi, dim3(elem_blocks((size_t)nloops * s.N * s.H)), dim3(256), 0, hs, s, w.U, u);
    return last_error();
}

int loop_set_resident(int mode) {
    if (mode < 0 || mode > 2) return LOOP_EINVAL;
    return g_resident.exchange(mode);
}

int loop_resident_supported(int Nx, int Ns) {
    if (check_shape(22.0, Nx, Ns, 1)) return 0;
    return resident_usable(Nx, Ns) ? 1 : 0;
}

int loop_step_form(int Nx, int Ns, int nloops) {
    if (check_shape(22.0, Nx, Ns, nloops)) return LOOP_EINVAL;
    const int mode = g_resident.load();
    return (mode != 0 && resident_usable(Nx, Ns) && (mode == 2 || resident_preferred(Nx, Ns, nloops))) ? 1 : 0;
}

int loop_update(double L, int Nx, int Ns, int nloops, double* T, double* uhat, const double* Ghat,
                const double* dJdT, double dtau, int scheme, void* stream) {
    int st = check_shape(L, Nx, Ns, nloops);
    if (st) return st;
    if (!aligned(T, 8) || !aligned(uhat, 16) || !aligned(Ghat, 16) || !aligned(dJdT, 8) ||
        (const void*)uhat == (const void*)Ghat)
        return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1)) return LOOP_EINVAL;
    Shape s = make_shape(L, Nx, Ns, nloops);
    hipStream_t hs = (hipStream_t)stream;
    hipLaunchKernelGGL(k_update, dim3(elem_blocks((size_t)s.nloops * s.N * s.H)), dim3(256), 0, hs, s, T,
                       reinterpret_cast<cd*>(uhat), reinterpret_cast<const cd*>(Ghat), dtau, scheme);
    hipLaunchKernelGGL(k_update_T, dim3((nloops + 255) / 256), dim3(256), 0, hs, nloops, T, dJdT, dtau);
    return last_error();
}

int loop_batch_create(int nloops, const double* L, const int* Nx, const int* Ns, void** plan) {
    if (!plan || !L || !Nx || !Ns || nloops < 1 || nloops > 65535) return LOOP_EINVAL;
    *plan = nullptr;
    for (int l = 0; l < nloops; ++l) {
        const int st = check_shape(L[l], Nx[l], Ns[l], 1);
        if (st) return st;
        if (Nx[l] > 512) return LOOP_ENOTSUP;  // batched row passes take Nx <= 512
    }
    const cd* tw;
    int st = get_table(&tw);
    if (st) return st;
    BatchPlan* p = new BatchPlan();
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return LOOP_EHIP;
    }
    p->nloops = nloops;
    p->loops.resize(nloops);
    // work space: header | queue | done[nloops] | per-loop regions
    size_t off = round_up(sizeof(WsHeader));
    p->q_off = off;
    off = round_up(off + sizeof(BatchQueue));
    p->done_off = off;
    off = round_up(off + sizeof(int) * (size_t)nloops);
    size_t pool = 0;
    for (int l = 0; l < nloops; ++l) {
        BatchLoop& b = p->loops[l];
        b.sh = make_shape(L[l], Nx[l], Ns[l], 1);
        Work w{};
        const size_t sz = layout(b.sh, reinterpret_cast<char*>(off), &w);
        const size_t base = off;
        auto rel = [&](const void* q) { return (size_t)reinterpret_cast<uintptr_t>(q); };
        b.off = WsOff{rel(w.A), rel(w.BD), rel(w.Cb), rel(w.U), rel(w.G), rel(w.partial), rel(w.J), rel(w.dJdT),
                      rel(w.Told)};
        off = round_up(base + sz);
        b.uoff = pool;
        pool += (size_t)b.sh.N * b.sh.H;
        b.nt[PASS_A] = col_tiles(b.sh);
        b.nt[PASS_B] = row_tiles(b.sh);
        b.nt[PASS_C] = col_tiles(b.sh);
        b.nt[PASS_D] = row_tiles(b.sh);
        b.nt[PASS_E] = col_tiles(b.sh);
        b.ipl = b.nt[PASS_B] + b.nt[PASS_C] + b.nt[PASS_D] + b.nt[PASS_E];
        p->max_nb = std::max(p->max_nb, b.sh.NB);
        p->max_c = std::max(p->max_c, b.sh.C);
        p->max_n = std::max(p->max_n, b.sh.N);
        p->max_h = std::max(p->max_h, b.sh.H);
        p->lds_bytes = std::max(p->lds_bytes, pass_lds_bytes(b.sh));
        for (int pass = PASS_A; pass <= PASS_E; ++pass)
            for (int v = 0; v < rag_count(pass); ++v)
                p->pass_lds[pass][v] =
                    std::max(p->pass_lds[pass][v], rag_lds_bytes(b.sh, pass, rag_variant(pass, v).pt));
        p->min_m = std::min(p->min_m, b.sh.M);
        p->max_m = std::max(p->max_m, b.sh.M);
        p->min_n = std::min(p->min_n, b.sh.N);
        p->max_n2 = std::max(p->max_n2, b.sh.N);
    }
    for (int pass = PASS_A; pass <= PASS_E; ++pass) p->variant[pass] = rag_default(p, pass);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        const auto it = tune_cache().find(plan_signature(p));
        if (it != tune_cache().end()) {
            p->schedule = it->second.schedule;
            p->nstreams = it->second.nstreams;
            for (int pass = PASS_A; pass <= PASS_E; ++pass) p->variant[pass] = it->second.variant[pass];
        }
    }
    p->ws_bytes = off;
    p->pool_elems = pool;
    // item list: larger loops first within each pass, so that they start early
    std::vector<int> order(nloops);
    for (int l = 0; l < nloops; ++l) order[l] = l;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (size_t)p->loops[a].sh.M * p->loops[a].sh.N > (size_t)p->loops[b].sh.M * p->loops[b].sh.N;
    });
    // persistent schedule: each loop on one XCD (larger loops placed first, each on the XCD
    // with the fewest bytes per step so far), and one item list per XCD. The XCDs are those
    // whose XCC_IDs a probe launch of many blocks reports (blocks are dealt to every XCD).
    {
        int cus = 1;
        int* d_seen = nullptr;
        int seen[kMaxXcd] = {};
        const bool ok = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
                        hipMalloc((void**)&d_seen, sizeof(seen)) == hipSuccess &&
                        hipMemcpy(d_seen, seen, sizeof(seen), hipMemcpyHostToDevice) == hipSuccess;
        if (ok) hipLaunchKernelGGL(k_xcc_probe, dim3(16 * std::max(cus, 1)), dim3(64), 0, 0, d_seen);
        const bool ok2 = ok && hipGetLastError() == hipSuccess &&
                         hipMemcpy(seen, d_seen, sizeof(seen), hipMemcpyDeviceToHost) == hipSuccess;
        if (d_seen) hipFree(d_seen);
        if (!ok2) {
            free_plan(p);
            return LOOP_EHIP;
        }
        p->nxcd = 0;
        for (int id = 0; id < kMaxXcd; ++id) p->xlist[id] = seen[id] ? p->nxcd++ : -1;
        if (p->nxcd == 0) {
            free_plan(p);
            return LOOP_EHIP;
        }
    }
    std::vector<int> xcd_of(nloops, 0);
    {
        std::vector<size_t> load(p->nxcd, 0);
        for (int l : order) {
            const Shape& sh = p->loops[l].sh;
            int g = 0;
            for (int h = 1; h < p->nxcd; ++h)
                if (load[h] < load[g]) g = h;
            xcd_of[l] = g;
            load[g] += 9 * (size_t)sh.C * sh.N + 4 * (size_t)sh.C * sh.NB;
        }
    }
    std::vector<uint32_t> items;
    for (int x = 0; x < p->nxcd; ++x) {
        p->xoff[x] = (int)items.size();
        for (int l : order)
            if (xcd_of[l] == x)
                for (int t = 0; t < p->loops[l].nt[PASS_A]; ++t) items.push_back(item_code(l, PASS_A, t));
        p->nA[x] = (int)items.size() - p->xoff[x];
        for (int pass = PASS_B; pass <= PASS_E; ++pass)
            for (int l : order)
                if (xcd_of[l] == x)
                    for (int t = 0; t < p->loops[l].nt[pass]; ++t) items.push_back(item_code(l, pass, t));
        p->ips[x] = (int)items.size() - p->xoff[x] - p->nA[x];
    }
    // per-pass code lists for the launch-per-pass schedule
    std::vector<uint32_t> pcodes;
    for (int pass = PASS_A; pass <= PASS_E; ++pass) {
        p->pass_off[pass] = (int)pcodes.size();
        for (int l : order)
            for (int t = 0; t < p->loops[l].nt[pass]; ++t) pcodes.push_back(item_code(l, pass, t));
    }
    p->pass_off[5] = (int)pcodes.size();
    // multi-stream schedule: K groups of about equal bytes per step (larger loops placed first,
    // each on the lightest group so far), for K = 2, 3, 4
    std::vector<uint32_t> gcodes;
    for (int K = 2; K <= 4; ++K) {
        std::vector<int> group(nloops, 0);
        size_t load[4] = {0, 0, 0, 0};
        for (int l : order) {
            const Shape& sh = p->loops[l].sh;
            int g = 0;
            for (int h = 1; h < K; ++h)
                if (load[h] < load[g]) g = h;
            group[l] = g;
            load[g] += 9 * (size_t)sh.C * sh.N + 4 * (size_t)sh.C * sh.NB;
        }
        for (int g = 0; g < K; ++g)
            for (int pass = PASS_A; pass <= PASS_E; ++pass) {
                p->group_off[K - 2][g][pass] = (int)gcodes.size();
                for (int l : order)
                    if (group[l] == g)
                        for (int t = 0; t < p->loops[l].nt[pass]; ++t) gcodes.push_back(item_code(l, pass, t));
                p->group_off[K - 2][g][pass + 1] = (int)gcodes.size();
            }
    }
    // one resident wave of blocks
    int per_cu = 1, cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, kBlock, p->lds_bytes) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
        free_plan(p);
        return LOOP_EHIP;
    }
    p->grid = std::max(1, per_cu) * std::max(1, cus);
    if (hipMalloc((void**)&p->d_loops, sizeof(BatchLoop) * nloops) != hipSuccess ||
        hipMalloc((void**)&p->d_items, sizeof(uint32_t) * items.size()) != hipSuccess ||
        hipMemcpy(p->d_loops, p->loops.data(), sizeof(BatchLoop) * nloops, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_items, items.data(), sizeof(uint32_t) * items.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc((void**)&p->d_pass_codes, sizeof(uint32_t) * pcodes.size()) != hipSuccess ||
        hipMemcpy(p->d_pass_codes, pcodes.data(), sizeof(uint32_t) * pcodes.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMalloc((void**)&p->d_group_codes, sizeof(uint32_t) * gcodes.size()) != hipSuccess ||
        hipMemcpy(p->d_group_codes, gcodes.data(), sizeof(uint32_t) * gcodes.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess) {
        free_plan(p);
        return LOOP_EHIP;
    }
    for (int k = 0; k < 3; ++k)
        if (hipStreamCreateWithFlags(&p->sx[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_lag[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_join[k], hipEventDisableTiming) != hipSuccess) {
            free_plan(p);
            return LOOP_EHIP;
        }
    *plan = p;
    return LOOP_OK;
}

int loop_batch_set_schedule(void* plan, int schedule) {
    BatchPlan* p = static_cast<BatchPlan*>(plan);
    if (!p || schedule < LOOP_BATCH_PER_PASS || schedule > LOOP_BATCH_STREAMS) return LOOP_EINVAL;
    p->schedule = schedule;
    return LOOP_OK;
}

int loop_batch_destroy(void* plan) {
    free_plan(static_cast<BatchPlan*>(plan));
    return LOOP_OK;
}

int loop_batch_info(const void* plan, size_t* ws_bytes, size_t* pool_elems, long long* uhat_offsets) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    if (!p) return LOOP_EINVAL;
    if (ws_bytes) *ws_bytes = p->ws_bytes;
    if (pool_elems) *pool_elems = p->pool_elems;
    if (uhat_offsets)
        for (int l = 0; l < p->nloops; ++l) uhat_offsets[l] = (long long)p->loops[l].uoff;
    return LOOP_OK;
}

int loop_batch_workspace_init(const void* plan, void* ws, size_t ws_bytes, void* stream) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    if (!p || !aligned(ws, 256)) return LOOP_EINVAL;
    if (ws_bytes < p->ws_bytes) return LOOP_EWORKSPACE;
    hipStream_t hs = (hipStream_t)stream;
    char* base = static_cast<char*>(ws);
    hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(1), 0, hs, (WsHeader*)ws);
    hipLaunchKernelGGL(k_batch_ws_init, dim3((p->nloops + 255) / 256), dim3(256), 0, hs,
                       reinterpret_cast<BatchQueue*>(base + p->q_off), reinterpret_cast<int*>(base + p->done_off),
                       p->nloops);
    return last_error();
}

namespace {
int batch_check(const BatchPlan* p, const void* ws, size_t ws_bytes, const cd** tw) {
    if (!p || !aligned(ws, 256)) return LOOP_EINVAL;
    if (ws_bytes < p->ws_bytes) return LOOP_EWORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LOOP_EHIP;
    if (dev != p->device) return LOOP_EINVAL;
    return get_table(tw);
}

BatchArgs batch_args(const BatchPlan* p, char* base, double* T, double* J_hist, int nsteps, double dtau, int scheme,
                     const cd* tw) {
    BatchArgs a;
    a.loops = p->d_loops;
    a.items = p->d_items;
    a.nloops = p->nloops;
    for (int x = 0; x < kMaxXcd; ++x) {
        a.xlist[x] = p->xlist[x];
        a.xoff[x] = p->xoff[x];
        a.nA[x] = p->nA[x];
        a.ips[x] = p->ips[x];
    }
    a.nsteps = nsteps;
    a.q = reinterpret_cast<BatchQueue*>(base + p->q_off);
    a.done = reinterpret_cast<int*>(base + p->done_off);
    a.ws = base;
    a.status = reinterpret_cast<int*>(base);
    a.T = T;
    a.J_hist = J_hist;
    a.dtau = dtau;
    a.scheme = scheme;
    a.tw = tw;
    a.spin_ticks = (unsigned long long)(p->wait_limit * kWallClockHz);
    return a;
}

// One pass over the tiles c[0 .. n) with the plan's variant for that pass.
const char* rag_name(int pass, int v) {
    static const char* names[5][kRagVariants] = {
        {"k_rag<0, 0>", "k_rag<0, 1>", "k_rag<0, 2>", "k_rag<0, 3>"},
        {"k_rag<1, 0>", "k_rag<1, 1>", "k_rag<1, 2>", "k_rag<1, 3>"},
        {"k_rag<2, 0>", "k_rag<2, 1>", "k_rag<2, 2>", "k_rag<2, 3>"},
        {"k_rag<3, 0>", "k_rag<3, 1>", "k_rag<3, 2>", "k_rag<3, 3>"},
        {"k_rag<4, 0>", "k_rag<4, 1>", "k_rag<4, 2>", "k_rag<4, 3>"}};
    return names[pass][v];
}

void launch_pass_codes(const BatchPlan* p, int pass, int step, const BatchArgs& a, hipStream_t hs,
                       const uint32_t* c, int n) {
    if (n == 0) return;
    const dim3 grid(n);
    const int v = p->variant[pass];
    const size_t lds = p->pass_lds[pass][v];
    TraceScope ts_(rag_name(pass, v), 0, hs);
    switch (pass) {
        case PASS_A: launch_rag<PASS_A>(v, grid, lds, hs, a, c, step, ts_); break;
        case PASS_B: launch_rag<PASS_B>(v, grid, lds, hs, a, c, step, ts_); break;
        case PASS_C: launch_rag<PASS_C>(v, grid, lds, hs, a, c, step, ts_); break;
        case PASS_D: launch_rag<PASS_D>(v, grid, lds, hs, a, c, step, ts_); break;
        default: launch_rag<PASS_E>(v, grid, lds, hs, a, c, step, ts_); break;
    }
}

void launch_pass(const BatchPlan* p, int pass, int step, const BatchArgs& a, hipStream_t hs) {
    launch_pass_codes(p, pass, step, a, hs, p->d_pass_codes + p->pass_off[pass],
                      p->pass_off[pass + 1] - p->pass_off[pass]);
}

void launch_group_pass(const BatchPlan* p, int g, int pass, int step, const BatchArgs& a, hipStream_t hs) {
    const int* off = p->group_off[p->nstreams - 2][g];
    launch_pass_codes(p, pass, step, a, hs, p->d_group_codes + off[pass], off[pass + 1] - off[pass]);
}

// Multi-stream schedule: group 0 on the caller's stream, group g > 0 on the plan's stream
// sx[g - 1], each group started one pass after the previous one (after its first pass B), so
// that the GPU runs different passes of different groups side by side, each as its own
// kernel with its own registers and LDS. Events fork the plan's streams from the caller's and
// join them back before the caller's next work. Returns LOOP_EHIP if an event could not be
// recorded or waited on: the groups' order would then not be guaranteed.
int launch_streams(const BatchPlan* p, int nsteps, const BatchArgs& a, hipStream_t hs) {
    const int K = p->nstreams;
    auto st = [&](int g) { return g == 0 ? hs : p->sx[g - 1]; };
    bool ok = hipEventRecord(p->ev_fork, hs) == hipSuccess;
    for (int g = 1; g < K; ++g) ok = ok && hipStreamWaitEvent(st(g), p->ev_fork, 0) == hipSuccess;
    if (!ok) return LOOP_EHIP;
    for (int g = 0; g < K; ++g) {
        if (g > 0 && hipStreamWaitEvent(st(g), p->ev_lag[g - 1], 0) != hipSuccess) return LOOP_EHIP;
        launch_group_pass(p, g, PASS_A, 0, a, st(g));
        launch_group_pass(p, g, PASS_B, 0, a, st(g));
        if (g + 1 < K && hipEventRecord(p->ev_lag[g], st(g)) != hipSuccess) return LOOP_EHIP;
    }
    // queue the groups' launches in turn, one pass each
    for (int i = 0; i < nsteps; ++i)
        for (int pass = PASS_B; pass <= PASS_E; ++pass)
            for (int g = 0; g < K; ++g)
                if (!(i == 0 && pass == PASS_B)) launch_group_pass(p, g, pass, i, a, st(g));
    for (int g = 1; g < K; ++g) {
        if (hipEventRecord(p->ev_join[g - 1], st(g)) != hipSuccess ||
            hipStreamWaitEvent(hs, p->ev_join[g - 1], 0) != hipSuccess)
            return LOOP_EHIP;
    }
    return LOOP_OK;
}
}  // namespace

int loop_batch_load(const void* plan, const double* uhat_pool, void* ws, size_t ws_bytes, void* stream) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    const cd* tw;
    int st = batch_check(p, ws, ws_bytes, &tw);
    if (st) return st;
    if (!aligned(uhat_pool, 16)) return LOOP_EINVAL;
    TraceScope ts_("k_to_band_batch", 0, (hipStream_t)stream);
    ts_.launch(k_to_band_batch, dim3((p->max_nb + 31) / 32, (p->max_c + 31) / 32, p->nloops), dim3(256), 0,
                       (hipStream_t)stream, p->d_loops, reinterpret_cast<const cd*>(uhat_pool), static_cast<char*>(ws));
    return last_error();
}

int loop_batch_store(const void* plan, double* uhat_pool, void* ws, size_t ws_bytes, void* stream) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    const cd* tw;
    int st = batch_check(p, ws, ws_bytes, &tw);
    if (st) return st;
    if (!aligned(uhat_pool, 16)) return LOOP_EINVAL;
    TraceScope ts_("k_from_band_batch", 0, (hipStream_t)stream);
    ts_.launch(k_from_band_batch, dim3((p->max_n + 31) / 32, (p->max_h + 31) / 32, p->nloops), dim3(256), 0,
                       (hipStream_t)stream, p->d_loops, static_cast<const char*>(ws), reinterpret_cast<cd*>(uhat_pool));
    return last_error();
}

int loop_batch_pass(const void* plan, int pass, int step, int nsteps, double* T, double dtau, int scheme,
                    double* J_hist, void* ws, size_t ws_bytes, void* stream) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    const cd* tw;
    int st = batch_check(p, ws, ws_bytes, &tw);
    if (st) return st;
    if (pass < PASS_A || pass > PASS_E || nsteps < 1 || step < 0 || step >= nsteps || !aligned(T, 8) ||
        (J_hist && !aligned(J_hist, 8)))
        return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1)) return LOOP_EINVAL;
    const BatchArgs a = batch_args(p, static_cast<char*>(ws), T, J_hist, nsteps, dtau, scheme, tw);
    launch_pass(p, pass, step, a, (hipStream_t)stream);
    return last_error();
}

int loop_batch_step(const void* plan, double* T, double* uhat_pool, double dtau, int scheme, int nsteps,
                    double* J_hist, void* ws, size_t ws_bytes, void* stream) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    if (!p || !aligned(T, 8) || !aligned(uhat_pool, 16) || (J_hist && !aligned(J_hist, 8))) return LOOP_EINVAL;
    if (!(dtau > 0.0) || !std::isfinite(dtau) || (scheme != 0 && scheme != 1) || nsteps < 0) return LOOP_EINVAL;
    const cd* tw;
    int st = batch_check(p, ws, ws_bytes, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    char* base = static_cast<char*>(ws);
    if ((st = loop_batch_load(plan, uhat_pool, ws, ws_bytes, stream))) return st;
    if (nsteps > 0) {
        const BatchArgs a = batch_args(p, base, T, J_hist, nsteps, dtau, scheme, tw);
        if (p->schedule == LOOP_BATCH_PERSISTENT) {
            for (int x = 0; x < p->nxcd; ++x)
                if ((long long)p->nA[x] + (long long)nsteps * p->ips[x] >= (1ll << 31)) return LOOP_EINVAL;
            hipLaunchKernelGGL(k_batch_reset, dim3((p->nloops + 255) / 256), dim3(256), 0, hs, a.q, a.done, p->nloops);
            TraceScope ts_("k_batch", 0, hs);
            ts_.launch(k_batch, dim3(p->grid), dim3(kBlock), p->lds_bytes, hs, a);
        } else if (p->schedule == LOOP_BATCH_STREAMS) {
            if ((st = launch_streams(p, nsteps, a, hs))) return st;
        } else {
            launch_pass(p, PASS_A, 0, a, hs);
            for (int i = 0; i < nsteps; ++i)
                for (int pass = PASS_B; pass <= PASS_E; ++pass) launch_pass(p, pass, i, a, hs);
        }
    }
    return loop_batch_store(plan, uhat_pool, ws, ws_bytes, stream);
}

int loop_batch_set_wait_limit(void* plan, double seconds) {
    BatchPlan* p = static_cast<BatchPlan*>(plan);
    if (!p || !(seconds >= 0.0) || !(seconds <= 3600.0)) return LOOP_EINVAL;
    p->wait_limit = seconds;
    return LOOP_OK;
}

int loop_batch_set_streams(void* plan, int nstreams) {
    BatchPlan* p = static_cast<BatchPlan*>(plan);
    if (!p || nstreams < 2 || nstreams > 4) return LOOP_EINVAL;
    p->nstreams = nstreams;
    return LOOP_OK;
}

int loop_batch_set_variant(void* plan, int pass, int variant) {
    BatchPlan* p = static_cast<BatchPlan*>(plan);
    if (!p || pass < PASS_A || pass > PASS_E || !rag_covers(p, pass, variant)) return LOOP_EINVAL;
    p->variant[pass] = variant;
    return LOOP_OK;
}

int loop_batch_get_config(const void* plan, int* schedule, int* variants, int* nstreams) {
    const BatchPlan* p = static_cast<const BatchPlan*>(plan);
    if (!p) return LOOP_EINVAL;
    if (schedule) *schedule = p->schedule;
    if (nstreams) *nstreams = p->nstreams;
    if (variants)
        for (int pass = PASS_A; pass <= PASS_E; ++pass) variants[pass] = p->variant[pass];
    return LOOP_OK;
}

int loop_batch_autotune(void* plan, const double* T, const double* uhat_pool, int reps, double* report, void* ws,
                        size_t ws_bytes, void* stream) {
    BatchPlan* p = static_cast<BatchPlan*>(plan);
    if (!p || !aligned(T, 8) || !aligned(uhat_pool, 16) || reps < 1 || reps > 1000) return LOOP_EINVAL;
    // The kernels' work does not depend on the step size or the scheme, so the timing runs
    // take a step too small to move the state: repeated passes and steps stay finite.
    const double dtau = 1e-30;
    const int scheme = LOOP_EULER_IMEX;
    const cd* tw;
    int st = batch_check(p, ws, ws_bytes, &tw);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    char* base = static_cast<char*>(ws);
    double* tT = nullptr;
    double* tpool = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (tT) hipFree(tT);
        if (tpool) hipFree(tpool);
    };
    const size_t pool_bytes = sizeof(cd) * p->pool_elems;
    if (hipMalloc((void**)&tT, sizeof(double) * p->nloops) != hipSuccess ||
        hipMalloc((void**)&tpool, pool_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess ||
        hipMemcpyAsync(tT, T, sizeof(double) * p->nloops, hipMemcpyDeviceToDevice, hs) != hipSuccess ||
        hipMemcpyAsync(tpool, uhat_pool, pool_bytes, hipMemcpyDeviceToDevice, hs) != hipSuccess) {
        release();
        return LOOP_EHIP;
    }
    std::vector<double> rep(5 * kRagVariants + 5, -1.0);
    // Mean microseconds per call of `launch` over n back-to-back calls, best of three trials.
    // A failed event call marks the run (timed_ok), and the tuner then reports LOOP_EHIP.
    bool timed_ok = true;
    auto time_calls = [&](auto&& launch, int n) -> double {
        double best = 1e300;
        for (int trial = 0; trial < 3; ++trial) {
            timed_ok = timed_ok && hipEventRecord(e0, hs) == hipSuccess;
            for (int i = 0; i < n; ++i) launch();
            float ms = 0.0f;
            timed_ok = timed_ok && hipEventRecord(e1, hs) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                       hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            best = std::min(best, 1e3 * (double)ms / n);
        }
        return best;
    };
    // Every pass is a function of the work space alone (pass D also moves the copy of T), so
    // after one full step each pass can be repeated in place and timed.
    loop_batch_load(p, tpool, ws, ws_bytes, stream);
    const BatchArgs a = batch_args(p, base, tT, nullptr, 2, dtau, scheme, tw);
    for (int pass = PASS_A; pass <= PASS_E; ++pass) launch_pass(p, pass, 0, a, hs);
    for (int pass = PASS_A; pass <= PASS_E; ++pass) {
        const int incumbent = p->variant[pass];
        int best_v = incumbent;
        double best_t = 1e300;
        for (int v = 0; v < rag_count(pass); ++v) {
            if (!rag_covers(p, pass, v)) continue;
            p->variant[pass] = v;
            launch_pass(p, pass, 0, a, hs);  // the first launch of a kernel also loads its code
            const double t = time_calls([&] { launch_pass(p, pass, 0, a, hs); }, reps);
            rep[pass * kRagVariants + v] = t;
            if (t < best_t) {
                best_t = t;
                best_v = v;
            }
        }
        // the plan's current variant stays unless another is faster by more than 1%, so that
        // timing noise between near-equal variants does not flip the choice from run to run
        const double t_inc = rep[pass * kRagVariants + incumbent];
        if (best_v != incumbent && t_inc > 0.0 && best_t > 0.99 * t_inc) best_v = incumbent;
        p->variant[pass] = best_v;
    }
    // schedules: per-pass, then the multi-stream one with 2, 3 and 4 streams. The persistent
    // schedule is not timed: it measured 3-5x slower than these on every workload (an
    // agent-scope release per item to order work across the XCDs' separate L2 caches).
    double best_us = 1e300;
    int best_s = LOOP_BATCH_PER_PASS, best_k = 2;
    for (int c = 0; c < 5; ++c) {
        if (c == 1) continue;  // persistent: reported as -1
        const int sc = c < 2 ? c : LOOP_BATCH_STREAMS, k = c < 2 ? 2 : c;
        p->schedule = sc;
        p->nstreams = k;
        timed_ok = timed_ok && loop_batch_step(p, tT, tpool, dtau, scheme, 1, nullptr, ws, ws_bytes, stream) == 0;
        const double us = time_calls(
                              [&] {
                                  timed_ok = timed_ok && loop_batch_step(p, tT, tpool, dtau, scheme, reps, nullptr,
                                                                         ws, ws_bytes, stream) == 0;
                              },
                              1) /
                          reps;
        rep[5 * kRagVariants + c] = us;
        if (us < best_us) {
            best_us = us;
            best_s = sc;
            best_k = k;
        }
    }
    p->schedule = best_s;
    p->nstreams = best_k;
    st = last_error();
    if (hipStreamSynchronize(hs) != hipSuccess || !timed_ok) st = LOOP_EHIP;
    release();
    if (st) return st;
    st = loop_status_sync(ws, stream);
    if (st) return st;
    if (report) std::copy(rep.begin(), rep.end(), report);
    TunedConfig c;
    c.schedule = p->schedule;
    c.nstreams = p->nstreams;
    for (int pass = PASS_A; pass <= PASS_E; ++pass) c.variant[pass] = p->variant[pass];
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache()[plan_signature(p)] = c;
    return LOOP_OK;
}

int loop_trace_start(void) {
    std::lock_guard<std::mutex> g(g_trace_mu);
    for (auto& r : g_trace_recs) {
        g_trace_pool.push_back(r.a);
        g_trace_pool.push_back(r.b);
    }
    g_trace_recs.clear();
    g_trace_stats.clear();
    g_trace_failed = false;
    g_trace_on.store(1);
    return LOOP_OK;
}

int loop_trace_stop(void) {
    g_trace_on.store(0);
    std::lock_guard<std::mutex> g(g_trace_mu);
    std::map<std::string, TraceStat> acc;
    std::vector<std::string> order;
    bool ok = !g_trace_failed;
    for (auto& r : g_trace_recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            ok = false;
        } else {
            if (!acc.count(r.name)) order.push_back(r.name);
            TraceStat& t = acc[r.name];
            const double us = 1e3 * (double)ms;
            t.launches += 1;
            t.total_us += us;
            t.min_us = std::min(t.min_us, us);
            t.max_us = std::max(t.max_us, us);
        }
        g_trace_pool.push_back(r.a);
        g_trace_pool.push_back(r.b);
    }
    g_trace_recs.clear();
    g_trace_stats.clear();
    for (const auto& n : order) g_trace_stats.emplace_back(n, acc[n]);
    return ok ? LOOP_OK : LOOP_EHIP;
}

int loop_trace_count(void) {
    std::lock_guard<std::mutex> g(g_trace_mu);
    return (int)g_trace_stats.size();
}

int loop_trace_get(int i, char* name, int name_len, long long* launches, double* total_us, double* min_us,
                   double* max_us) {
    std::lock_guard<std::mutex> g(g_trace_mu);
    if (i < 0 || i >= (int)g_trace_stats.size() || !name || name_len < 1) return LOOP_EINVAL;
    const auto& e = g_trace_stats[i];
    std::strncpy(name, e.first.c_str(), (size_t)name_len - 1);
    name[name_len - 1] = 0;
    if (launches) *launches = e.second.launches;
    if (total_us) *total_us = e.second.total_us;
    if (min_us) *min_us = e.second.min_us;
    if (max_us) *max_us = e.second.max_us;
    return LOOP_OK;
}

int loop_status_sync(void* ws, void* stream) {
    if (!aligned(ws, 256)) return LOOP_EINVAL;
    WsHeader h;
    hipStream_t hs = (hipStream_t)stream;
    if (hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, hs) != hipSuccess) return LOOP_EHIP;
    if (hipStreamSynchronize(hs) != hipSuccess) return LOOP_EHIP;
    if (h.magic != kWsMagic) return LOOP_EWORKSPACE;
    if (h.status != 0) {
        hipLaunchKernelGGL(k_ws_clear_status, dim3(1), dim3(1), 0, hs, (WsHeader*)ws);
        if (last_error()) return LOOP_EHIP;
    }
    return h.status;
}

const char* loop_status_string(int status) {
    switch (status) {
        case LOOP_OK: return "ok";
        case LOOP_EINVAL: return "invalid argument";
        case LOOP_ENOTSUP: return "unsupported size";
        case LOOP_EHIP: return "HIP runtime error";
        case LOOP_ENONFINITE: return "non-finite or non-positive period or cost on device";
        case LOOP_EWORKSPACE: return "work space too small or not initialised";
        case LOOP_EHANG: return "batched scheduler dependency wait timed out";
        default: return "unknown status";
    }
}

}  // extern "C"
