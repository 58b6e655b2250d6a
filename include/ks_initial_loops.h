/* ks_initial_loops.h - C ABI of the initial-loop pipeline (Sec. 4.3 of Azimi, Ashtari &
 * Schneider, arXiv:2007.06427), part of the same MI355X (gfx950) library as looporbit.h.
 *
 * Initial loops for the loop dynamics are cut from chaotic runs of the Kuramoto-Sivashinsky
 * equation u_t = -u u_x - u_xx - u_xxxx on [0, L) (eq. KS): the runs record the norm
 * ||u||(t) = sqrt(int_0^L u^2 dx) (eq. conventinal_L2norm); two maxima of it at t_a < t_b with
 * nearly equal values mark a segment; the segment, Fourier-transformed in time with its high
 * temporal frequencies dropped, is the field of a loop with period T = t_b - t_a.
 *
 * Conventions of looporbit.h hold: device pointers owned by the caller, interleaved complex
 * doubles (16-byte aligned), work queued on `stream` (hipStream_t or NULL), no call
 * synchronises or allocates, argument checks on the host before anything is queued, and the
 * status codes of loop_status.
 *
 * Instantaneous fields use the rfft layout of one row: Nx/2 + 1 complex values, element j =
 * u_hat_j of u(x_m) = sum_j u_hat_j e^{2 pi i j m / Nx} (forward-normalised). Runs keep the
 * two-thirds band |j| <= (Nx-1)/3; entries beyond it are ignored on input and written as 0.
 */
#ifndef KS_INITIAL_LOOPS_H
#define KS_INITIAL_LOOPS_H

#include "looporbit.h"

#ifdef __cplusplus
extern "C" {
#endif

/* nsteps ETDRK4 steps (Cox & Matthews 2002) of ntraj independent runs of eq. KS on the
 * Fourier-Galerkin system with the two-thirds rule: u_hat_j' = c_j u_hat_j + N_hat_j,
 * c_j = q_j^2 - q_j^4, N_hat = -(i q_j / 2) (u^2)_hat_j, q_j = 2 pi j / L, step dt. The
 * ETDRK4 coefficients are formed from phi-functions of dt c_j (series for |dt c_j| < 1).
 *   uhat   (ntraj, Nx/2 + 1) complex, in place: the runs' states.
 *   symmetric != 0: the centre-symmetric subspace u(-x) = -u(x) (eq. KS_sym): the state is
 *          projected onto odd fields (Re u_hat_j = 0) on input and after every step.
 *   sample_every: samples are taken of the states before steps 0, s, 2s, ..., nsteps - s
 *          (nsteps a multiple of s): nsamples = nsteps / s of them.
 *   norms  NULL, or (ntraj, sample_stride) doubles: norms[r * sample_stride + i] = ||u|| of
 *          run r at sample i.
 *   snaps  NULL, or (ntraj, sample_stride, Nx/2 + 1) complex: the sampled states.
 * Calls chain: the state left in uhat is the one the next call's sample 0 records, so the
 * caller can advance runs in pieces, offsetting norms/snaps by the samples already taken.
 * Nx: 16, 32, 64, 128 or 256 (LOOP_ENOTSUP for other powers of two in [8, 1024]).
 * LOOP_EINVAL: L or dt not positive and finite, ntraj outside [1, 2^20], nsteps < 0,
 * sample_every < 1 or not dividing nsteps, sample_stride < nsamples with an output given,
 * misaligned pointers. */
int ks_integrate(double L, int Nx, int ntraj, int symmetric, double dt, int nsteps, int sample_every, double* uhat,
                 double* norms, double* snaps, int sample_stride, void* stream);

/* Recurrences of the norm (Sec. 4.3): per run, every pair of maxima a < b of n_i =
 * norms[r * sample_stride + i], i < nsamples, with Tmin <= (b - a) dt_s <= Tmax and
 * |n_b - n_a| <= rel_tol n_a. A maximum is a sample 0 < i < nsamples - 1 with
 * n_{i-1} < n_i >= n_{i+1}. Pairs go to pairs[(r * cap + p) * 2 + {0, 1}] = (a, b) in
 * increasing (a, b); counts[r] receives the number of pairs found, of which the first
 * min(count, cap) are stored. Every decision is a comparison of values formed as written
 * here in IEEE double, so results are exact. pairs: (ntraj, cap, 2) int, 8-byte aligned;
 * counts: ntraj int. LOOP_EINVAL: ntraj outside [1, 2^20], nsamples < 0, sample_stride <
 * nsamples, cap < 0, dt_s not positive and finite, rel_tol negative or not finite, NaN
 * Tmin or Tmax, missing or misaligned pointers. */
int ks_recurrences(int ntraj, int nsamples, const double* norms, int sample_stride, double dt_s, double rel_tol,
                   double Tmin, double Tmax, int cap, int* pairs, int* counts, void* stream);

/* Loops from segments (Sec. 4.3): for loop l, triples[3 l .. 3 l + 2] = (run r, a, b)
 * selects samples a .. b - 1 of run r in snaps (layout of ks_integrate, with nsamples valid
 * samples per run). With n = b - a, the segment is read as one period of a field on
 * s_i = i / n; its temporal modes
 *   c_{j,k} = (1/n) sum_i u_hat_j(t_{a+i}) e^{-2 pi i k i / n},  |k| <= kc, j <= (Nx-1)/3,
 * are kept and everything else is dropped: uhat_loops (nloops, Ns, Nx/2 + 1) complex receives
 * the loops in the rfft layout of looporbit.h (row k mod Ns), T_loops[l] = n dt_s. A triple
 * with r outside [0, ntraj), a < 0, b > nsamples or n <= 2 kc gives a zero loop and T = 0.
 * LOOP_EINVAL: Nx or Ns not a power of two in [8, 1024], kc outside [0, (Ns-1)/3], nloops
 * outside [1, 65535], ntraj < 1, nsamples < 0, sample_stride < nsamples, dt_s not positive
 * and finite, missing or misaligned pointers. */
int ks_segments_to_loops(int Nx, int ntraj, int nsamples, const double* snaps, int sample_stride, int nloops,
                         const int* triples, double dt_s, int Ns, int kc, double* uhat_loops, double* T_loops,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif
