// Initial loops from chaotic Kuramoto-Sivashinsky runs (Sec. 4.3): the KS equation
// u_t = -u u_x - u_xx - u_xxxx (eq. KS) integrated by ETDRK4 on its Fourier-Galerkin system,
// the norm ||u||(t) (eq. conventinal_L2norm) recorded along the runs, pairs of its maxima
// that nearly repeat, and the temporal low-pass that turns a segment into a loop.
//
// One wavefront advances one run: a run's state is a few dozen modes, so the whole state,
// the ETDRK4 coefficients and the stage values stay in registers, and the two transforms of
// each nonlinear evaluation are direct sums through LDS (the band and the grid of one run
// fit in a few KB). Thousands of runs fill the chip; HBM sees only the samples.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ks_initial_loops.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct cd {
    double x, y;
};

// ----------------------------------------------------------------------------- ETDRK4
// phi_1..3 of z (phi_k(z) = sum_n z^n / (n + k)!): the series below |z| = 1, the recurrence
// phi_{k+1} = (phi_k - 1/k!) / z from phi_0 = e^z above (no cancellation worse than a factor
// of a few there).
__device__ void phis(double z, double& p1, double& p2, double& p3) {
    if (fabs(z) < 1.0) {
        // Horner over n = 24 .. 0 of z^n / (n + k)!, with 1/(n + k)! formed downwards
        double f = 1.0;  // 1/27!, built upwards once
        for (int i = 2; i <= 27; ++i) f /= (double)i;
        double inv[28];
        inv[27] = f;
        for (int i = 27; i >= 1; --i) inv[i - 1] = inv[i] * (double)i;
        double a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int n = 24; n >= 0; --n) {
            a1 = a1 * z + inv[n + 1];
            a2 = a2 * z + inv[n + 2];
            a3 = a3 * z + inv[n + 3];
        }
        p1 = a1;
        p2 = a2;
        p3 = a3;
    } else {
        p1 = expm1(z) / z;
        p2 = (p1 - 1.0) / z;
        p3 = (p2 - 0.5) / z;
    }
}

struct Etd {
    double E, E2, Q, f1, f2, f3, q;
};

// Coefficients of mode j (Cox & Matthews): z = h c_j, c_j = q^2 - q^4,
// Q = (h/2) phi_1(z/2), f1 = h (phi_1 - 3 phi_2 + 4 phi_3), f2 = h (phi_2 - 2 phi_3),
// f3 = h (4 phi_3 - phi_2).
__device__ Etd etd_coeffs(int j, double L, double h) {
    Etd e;
    e.q = kTwoPi * j / L;
    const double q2 = e.q * e.q;
    const double c = q2 - q2 * q2;
    const double z = h * c;
    double p1, p2, p3, h1, h2, h3;
    phis(z, p1, p2, p3);
    phis(0.5 * z, h1, h2, h3);
    e.E = exp(z);
    e.E2 = exp(0.5 * z);
    e.Q = 0.5 * h * h1;
    e.f1 = h * (p1 - 3.0 * p2 + 4.0 * p3);
    e.f2 = h * (p2 - 2.0 * p3);
    e.f3 = h * (4.0 * p3 - p2);
    return e;
}

// Per-run LDS: the band spectrum (K+1 complex), the grid (NX reals), the twiddles
// e^{2 pi i m / NX} (NX complex), and the partial sums of the forward transform.
// The forward transform is split into S segments of the grid per mode, so that S (K+1)
// lanes share its NX (K+1) terms instead of K+1 lanes.
template <int NX>
struct Dns {
    static constexpr int K = (NX - 1) / 3;
    static constexpr int H = NX / 2 + 1;
    static constexpr int R = (K + 1 + 63) / 64;  // modes per lane
    static constexpr int P = (NX + 63) / 64;     // grid points per lane
    static constexpr int S = (2 * (K + 1) <= 64) ? (4 * (K + 1) <= 64 ? (8 * (K + 1) <= 64 ? 8 : 4) : 2) : 1;
    static constexpr int SEG = NX / S;           // grid points per segment
    static constexpr int WI = S * (K + 1);       // (segment, mode) partial sums
    static constexpr int RF = (WI + 63) / 64;    // partial sums per lane
};

// N_hat_j = -(i q_j / 2) FFT(u^2)_j for the lane's modes, from the lane's band values v.
template <int NX>
__device__ __forceinline__ void nonlinear(const cd (&v)[Dns<NX>::R], const Etd (&co)[Dns<NX>::R], cd (&out)[Dns<NX>::R],
                                          cd* spec, double* grid, const cd* tw, cd* part) {
    using D = Dns<NX>;
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < D::R; ++r) {
        const int j = lane + 64 * r;
        if (j <= D::K) spec[j] = v[r];
    }
    __syncthreads();
    // grid values u(x_m) = Re u_0 + 2 sum_{j=1..K} Re(u_j e^{2 pi i j m / NX}), squared
#pragma unroll
    for (int p = 0; p < D::P; ++p) {
        const int m = lane + 64 * p;
        if (m < NX) {
            double s = 0.0;
            for (int j = 1; j <= D::K; ++j) {
                const cd a = spec[j];
                const cd w = tw[(j * m) & (NX - 1)];
                s += a.x * w.x - a.y * w.y;
            }
            const double u = spec[0].x + 2.0 * s;
            grid[m] = u * u;
        }
    }
    __syncthreads();
    // W_j = (1/NX) sum_m grid_m e^{-2 pi i j m / NX}: partial sums over segments of m, then
    // their sum in segment order; N_j = -(i q_j / 2) W_j
#pragma unroll
    for (int rr = 0; rr < D::RF; ++rr) {
        const int wi = lane + 64 * rr;
        if (wi < D::WI) {
            const int sg = wi / (D::K + 1), j = wi % (D::K + 1);
            double wx = 0.0, wy = 0.0;
            for (int m = sg * D::SEG; m < (sg + 1) * D::SEG; ++m) {
                const double g = grid[m];
                const cd w = tw[(j * m) & (NX - 1)];
                wx += g * w.x;
                wy -= g * w.y;
            }
            part[wi] = cd{wx, wy};
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < D::R; ++r) {
        const int j = lane + 64 * r;
        double wx = 0.0, wy = 0.0;
        if (j <= D::K) {
#pragma unroll
            for (int sg = 0; sg < D::S; ++sg) {
                const cd pw = part[sg * (D::K + 1) + j];
                wx += pw.x;
                wy += pw.y;
            }
        }
        const double s = 0.5 * co[r].q / NX;
        out[r] = cd{s * wy, -s * wx};
    }
    __syncthreads();  // spec, grid and the partial sums are free for the next evaluation
}

template <int NX>
__device__ __forceinline__ void record(int lane, const cd (&u)[Dns<NX>::R], double L, size_t row, double* norms,
                                       cd* snaps) {
    using D = Dns<NX>;
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < D::R; ++r) {
        const int j = lane + 64 * r;
        if (j <= D::K) e += (j == 0 ? 1.0 : 2.0) * (u[r].x * u[r].x + u[r].y * u[r].y);
    }
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if (norms && lane == 0) norms[row] = sqrt(L * e);
    if (snaps) {
        cd* s = snaps + row * D::H;
        for (int j = lane; j < D::H; j += 64) {
            cd x{0.0, 0.0};
#pragma unroll
            for (int r = 0; r < D::R; ++r)
                if (j == lane + 64 * r && j <= D::K) x = u[r];
            s[j] = x;
        }
    }
}

// One block (one wavefront) per run: nsteps ETDRK4 steps of run blockIdx.x.
template <int NX>
__global__ __launch_bounds__(64) void k_ks_etdrk4(double L, int sym, double h, int nsteps, int every, cd* uhat,
                                                  double* norms, cd* snaps, int stride) {
    using D = Dns<NX>;
    __shared__ cd spec[D::K + 1];
    __shared__ double grid[NX];
    __shared__ cd tw[NX];
    __shared__ cd part[D::WI];
    const int lane = threadIdx.x;
    const size_t run = blockIdx.x;
    for (int m = lane; m < NX; m += 64) {
        double s, c;
        sincospi(2.0 * m / NX, &s, &c);
        tw[m] = cd{c, s};
    }
    Etd co[D::R];
    cd u[D::R];
    cd* ur = uhat + run * D::H;
#pragma unroll
    for (int r = 0; r < D::R; ++r) {
        const int j = lane + 64 * r;
        co[r] = etd_coeffs(j <= D::K ? j : 0, L, h);
        u[r] = j <= D::K ? ur[j] : cd{0.0, 0.0};
        if (sym) u[r].x = 0.0;
    }
    __syncthreads();
    for (int i = 0; i < nsteps; ++i) {
        if (i % every == 0) record<NX>(lane, u, L, run * (size_t)stride + i / every, norms, snaps);
        cd Nu[D::R], Na[D::R], Nb[D::R], Nc[D::R], a[D::R], b[D::R], c[D::R];
        nonlinear<NX>(u, co, Nu, spec, grid, tw, part);
#pragma unroll
        for (int r = 0; r < D::R; ++r)
            a[r] = cd{co[r].E2 * u[r].x + co[r].Q * Nu[r].x, co[r].E2 * u[r].y + co[r].Q * Nu[r].y};
        nonlinear<NX>(a, co, Na, spec, grid, tw, part);
#pragma unroll
        for (int r = 0; r < D::R; ++r)
            b[r] = cd{co[r].E2 * u[r].x + co[r].Q * Na[r].x, co[r].E2 * u[r].y + co[r].Q * Na[r].y};
        nonlinear<NX>(b, co, Nb, spec, grid, tw, part);
#pragma unroll
        for (int r = 0; r < D::R; ++r)
            c[r] = cd{co[r].E2 * a[r].x + co[r].Q * (2.0 * Nb[r].x - Nu[r].x),
                      co[r].E2 * a[r].y + co[r].Q * (2.0 * Nb[r].y - Nu[r].y)};
        nonlinear<NX>(c, co, Nc, spec, grid, tw, part);
#pragma unroll
        for (int r = 0; r < D::R; ++r) {
            const Etd& e = co[r];
            cd n;
            n.x = e.E * u[r].x + e.f1 * Nu[r].x + 2.0 * e.f2 * (Na[r].x + Nb[r].x) + e.f3 * Nc[r].x;
            n.y = e.E * u[r].y + e.f1 * Nu[r].y + 2.0 * e.f2 * (Na[r].y + Nb[r].y) + e.f3 * Nc[r].y;
            if (sym) n.x = 0.0;
            const int j = lane + 64 * r;
            u[r] = j <= D::K ? n : cd{0.0, 0.0};
        }
    }
    for (int j = lane; j < D::H; j += 64) {
        cd x{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < D::R; ++r)
            if (j == lane + 64 * r && j <= D::K) x = u[r];
        ur[j] = x;
    }
}

// ------------------------------------------------------------------------- recurrences
__device__ __forceinline__ bool is_max(const double* n, int i, int ns) {
    return i >= 1 && i <= ns - 2 && n[i - 1] < n[i] && n[i] >= n[i + 1];
}

// pairs (a, b) of maxima of run blockIdx.x starting at maximum a, in increasing b; with
// out == nullptr only counted
__device__ int scan_from(const double* n, int a, int ns, double dt_s, double tol, double Tmin, double Tmax,
                         int2* out, int base, int cap) {
    int c = 0;
    for (int b = a + 1; b <= ns - 2; ++b) {
        const double T = (double)(b - a) * dt_s;
        if (T > Tmax) break;
        if (T >= Tmin && is_max(n, b, ns) && fabs(n[b] - n[a]) <= tol * n[a]) {
            if (out && base + c < cap) out[base + c] = make_int2(a, b);
            ++c;
        }
    }
    return c;
}

constexpr int kScanBlock = 256;

// One block per run. Tiles of 256 consecutive candidate samples a: each thread counts its
// pairs, an exclusive scan over the tile (in order of a) places them, then they are written.
__global__ __launch_bounds__(kScanBlock) void k_ks_recurrences(const double* norms, int stride, int ns, double dt_s,
                                                               double tol, double Tmin, double Tmax, int cap,
                                                               int2* pairs, int* counts) {
    __shared__ int sc[kScanBlock];
    __shared__ int base_s;
    const double* n = norms + (size_t)blockIdx.x * stride;
    int2* out = pairs + (size_t)blockIdx.x * cap;
    const int t = threadIdx.x;
    if (t == 0) base_s = 0;
    __syncthreads();
    for (int a0 = 0; a0 < ns; a0 += kScanBlock) {
        const int a = a0 + t;
        const bool m = a < ns && is_max(n, a, ns);
        const int c = m ? scan_from(n, a, ns, dt_s, tol, Tmin, Tmax, nullptr, 0, 0) : 0;
        sc[t] = c;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {  // inclusive Hillis-Steele scan
            const int v = t >= o ? sc[t - o] : 0;
            __syncthreads();
            sc[t] += v;
            __syncthreads();
        }
        const int base = base_s;
        if (m && c > 0) scan_from(n, a, ns, dt_s, tol, Tmin, Tmax, out, base + sc[t] - c, cap);
        __syncthreads();
        if (t == kScanBlock - 1) base_s = base + sc[t];
        __syncthreads();
    }
    if (t == 0) counts[blockIdx.x] = base_s;
}

// ------------------------------------------------------------------- segments to loops
// One block per loop; each thread forms loop entries (k, j) of the rfft layout:
// c_{j,k} = (1/n) sum_i u_hat_j(t_{a+i}) e^{-2 pi i k i / n} for |k| <= kc, j <= Kx, else 0.
__global__ __launch_bounds__(256) void k_ks_segments(const cd* snaps, int H, int ntraj, int ns, int stride,
                                                     const int* triples, double dt_s, int Ns, int kc, cd* loops,
                                                     double* T) {
    const int l = blockIdx.x;
    const int tr = triples[3 * l], a = triples[3 * l + 1], b = triples[3 * l + 2];
    const int n = b - a;
    const bool ok = tr >= 0 && tr < ntraj && a >= 0 && b <= ns && n > 2 * kc;
    const int Kx = (2 * (H - 1) - 1) / 3;
    cd* out = loops + (size_t)l * Ns * H;
    if (threadIdx.x == 0) T[l] = ok ? (double)n * dt_s : 0.0;
    const cd* seg = ok ? snaps + ((size_t)tr * stride + a) * H : nullptr;
    for (int e = threadIdx.x; e < Ns * H; e += blockDim.x) {
        const int row = e / H, j = e % H;
        const int k = row <= Ns / 2 ? row : row - Ns;
        cd v{0.0, 0.0};
        if (ok && j <= Kx && k >= -kc && k <= kc) {
            const long long km = ((long long)k % n + n) % n;
            double sx = 0.0, sy = 0.0;
            for (int i = 0; i < n; ++i) {
                const cd x = seg[(size_t)i * H + j];
                double s, c;
                sincospi(2.0 * (double)((km * i) % n) / n, &s, &c);  // e^{+2 pi i k i / n}
                sx += x.x * c + x.y * s;                              // x * conj(e)
                sy += x.y * c - x.x * s;
            }
            v = cd{sx / n, sy / n};
        }
        out[e] = v;
    }
}

bool pow2_size(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

int hip_status() { return hipGetLastError() == hipSuccess ? LOOP_OK : LOOP_EHIP; }

}  // namespace

extern "C" {

int ks_integrate(double L, int Nx, int ntraj, int symmetric, double dt, int nsteps, int sample_every, double* uhat,
                 double* norms, double* snaps, int sample_stride, void* stream) {
    if (!(L > 0.0) || !std::isfinite(L) || !(dt > 0.0) || !std::isfinite(dt)) return LOOP_EINVAL;
    if (ntraj < 1 || ntraj > 1 << 20 || nsteps < 0 || sample_every < 1 || nsteps % sample_every) return LOOP_EINVAL;
    if (Nx < 8 || Nx > 1024) return LOOP_EINVAL;
    if (!pow2_size(Nx, 16, 256)) return LOOP_ENOTSUP;
    if (!uhat || reinterpret_cast<uintptr_t>(uhat) % 16) return LOOP_EINVAL;
    const int ns = nsteps / sample_every;
    if ((norms || snaps) && sample_stride < ns) return LOOP_EINVAL;
    if ((norms && reinterpret_cast<uintptr_t>(norms) % 8) || (snaps && reinterpret_cast<uintptr_t>(snaps) % 16))
        return LOOP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    cd* u = reinterpret_cast<cd*>(uhat);
    cd* sn = reinterpret_cast<cd*>(snaps);
    const int sym = symmetric ? 1 : 0;
    switch (Nx) {
        case 16: hipLaunchKernelGGL(k_ks_etdrk4<16>, dim3(ntraj), dim3(64), 0, st, L, sym, dt, nsteps, sample_every, u, norms, sn, sample_stride); break;
        case 32: hipLaunchKernelGGL(k_ks_etdrk4<32>, dim3(ntraj), dim3(64), 0, st, L, sym, dt, nsteps, sample_every, u, norms, sn, sample_stride); break;
        case 64: hipLaunchKernelGGL(k_ks_etdrk4<64>, dim3(ntraj), dim3(64), 0, st, L, sym, dt, nsteps, sample_every, u, norms, sn, sample_stride); break;
        case 128: hipLaunchKernelGGL(k_ks_etdrk4<128>, dim3(ntraj), dim3(64), 0, st, L, sym, dt, nsteps, sample_every, u, norms, sn, sample_stride); break;
        case 256: hipLaunchKernelGGL(k_ks_etdrk4<256>, dim3(ntraj), dim3(64), 0, st, L, sym, dt, nsteps, sample_every, u, norms, sn, sample_stride); break;
    }
    return hip_status();
}

int ks_recurrences(int ntraj, int nsamples, const double* norms, int sample_stride, double dt_s, double rel_tol,
                   double Tmin, double Tmax, int cap, int* pairs, int* counts, void* stream) {
    if (ntraj < 1 || ntraj > 1 << 20 || nsamples < 0 || sample_stride < nsamples || cap < 0) return LOOP_EINVAL;
    if (!(dt_s > 0.0) || !std::isfinite(dt_s) || !(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return LOOP_EINVAL;
    if (std::isnan(Tmin) || std::isnan(Tmax)) return LOOP_EINVAL;
    if (!norms || !counts || (cap > 0 && !pairs) || reinterpret_cast<uintptr_t>(norms) % 8 ||
        reinterpret_cast<uintptr_t>(pairs) % 8 || reinterpret_cast<uintptr_t>(counts) % 4)
        return LOOP_EINVAL;
    hipLaunchKernelGGL(k_ks_recurrences, dim3(ntraj), dim3(kScanBlock), 0, (hipStream_t)stream, norms,
                       sample_stride, nsamples, dt_s, rel_tol, Tmin, Tmax, cap, reinterpret_cast<int2*>(pairs), counts);
    return hip_status();
}

int ks_segments_to_loops(int Nx, int ntraj, int nsamples, const double* snaps, int sample_stride, int nloops,
                         const int* triples, double dt_s, int Ns, int kc, double* uhat_loops, double* T_loops,
                         void* stream) {
    if (!pow2_size(Nx, 8, 1024) || !pow2_size(Ns, 8, 1024)) return LOOP_EINVAL;
    if (ntraj < 1 || nsamples < 0 || sample_stride < nsamples || nloops < 1 || nloops > 65535) return LOOP_EINVAL;
    if (kc < 0 || kc > (Ns - 1) / 3 || !(dt_s > 0.0) || !std::isfinite(dt_s)) return LOOP_EINVAL;
    if (!snaps || !triples || !uhat_loops || !T_loops || reinterpret_cast<uintptr_t>(snaps) % 16 ||
        reinterpret_cast<uintptr_t>(triples) % 4 || reinterpret_cast<uintptr_t>(uhat_loops) % 16 ||
        reinterpret_cast<uintptr_t>(T_loops) % 8)
        return LOOP_EINVAL;
    hipLaunchKernelGGL(k_ks_segments, dim3(nloops), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const cd*>(snaps), Nx / 2 + 1, ntraj, nsamples, sample_stride, triples, dt_s,
                       Ns, kc, reinterpret_cast<cd*>(uhat_loops), T_loops);
    return hip_status();
}

}  // extern "C"
