/* looporbit.h - C ABI of the MI355X (gfx950) library for one fictitious-time step of the
 * Kuramoto-Sivashinsky loop dynamics of the adjoint-based variational method
 * (Azimi, Ashtari & Schneider, arXiv:2007.06427).
 *
 * A loop l = [u(x, s); T] is a real field on x in [0, L), s in [0, 1), periodic in both, plus
 * its period T > 0 (Sec. 2, eq. loop_def). Its field is represented by Fourier coefficients
 * on an Nx x Ns grid (Sec. 4.2, eq. 2D_Fourier), truncated by the two-thirds rule in both
 * directions: |j| <= Kx = (Nx-1)/3 and |k| <= Ks = (Ns-1)/3, with integer division.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers are DEVICE pointers owned by the caller. Complex arrays are interleaved
 *   (re, im) doubles and must be 16-byte aligned; double arrays must be 8-byte aligned.
 * - Spectral layout ("rfft layout"): one loop occupies Ns * (Nx/2 + 1) complex values.
 *   Element [k][j] (row-major) holds u_hat_{j,k} for j = 0 .. Nx/2, with row k holding
 *   temporal mode k in FFT order (k < Ns/2 are the non-negative modes, k >= Ns/2 stand for
 *   k - Ns). This is the layout of a forward-normalised real-to-complex 2D transform of the
 *   real (Ns, Nx) grid. A batch of nloops loops of one shape is stored back to back.
 * - Inputs: entries outside the band are ignored. Column j = 0 is read through its
 *   Hermitian part (u_{0,k} + conj(u_{0,-k})) / 2, the column a real-valued inverse
 *   transform uses.
 * - Outputs: every entry of an output array is written, and entries outside the band are 0.
 * - J is HALF the paper's cost: J = 1/2 int_0^1 int_0^L r^2 dx ds. Then the paper's flow
 *   (eq. KS_G) is exactly G = -grad J in the inner product of eq. inner_product_definition.
 * - Results go to device memory and work is queued on `stream` (a hipStream_t, or NULL for
 *   the default stream). No call synchronises with the host, allocates, or frees memory,
 *   except that the first call on a device creates that device's twiddle table, and
 *   loop_status_sync waits for the stream. Every call may therefore be recorded into a HIP
 *   graph once the device is initialised (loop_init).
 * - Work space: `ws` is a caller-owned device buffer of at least loop_workspace_bytes(...)
 *   bytes, prepared once by loop_workspace_init. One work space per concurrently running
 *   stream. Calls that share a work space must be ordered on one stream.
 * - Errors: every call returns a loop_status. Argument checks run on the host before any
 *   work is queued. Nothing is queued when a check fails. Conditions that only the device
 *   can see (a non-finite or non-positive period, a non-finite cost) set a sticky status
 *   word in the work space, and loop_status_sync returns it.
 * - Sizes: Nx and Ns must be powers of two in [8, 1024]; 1 <= nloops <= 65535.
 */
#ifndef LOOPORBIT_H
#define LOOPORBIT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LOOP_OK = 0,
    LOOP_EINVAL = -1,      /* bad size, pointer, alignment, L, dtau or scheme */
    LOOP_ENOTSUP = -2,     /* a size or device the library does not support (e.g. Nx not a power of two) */
    LOOP_EHIP = -3,        /* a HIP runtime call failed */
    LOOP_ENONFINITE = -4,  /* device saw T <= 0 or a non-finite T or J (sticky, see loop_status_sync) */
    LOOP_EWORKSPACE = -5,  /* work space too small or not prepared by loop_workspace_init */
    LOOP_EHANG = -6        /* the batched scheduler's bounded dependency wait ran out (sticky) */
} loop_status;

typedef enum { LOOP_EULER_EXPLICIT = 0, LOOP_EULER_IMEX = 1 } loop_scheme;

/* Create this device's twiddle table (long-double accurate e^{-2 pi i t / 4096}). The current
 * HIP device is used. Calling it again is harmless. Must not be called under stream capture. */
int loop_init(void);

/* Release the tables of every device. */
int loop_shutdown(void);

/* Bytes of work space needed by a uniform batch of nloops loops of shape (Nx, Ns). */
int loop_workspace_bytes(int Nx, int Ns, int nloops, size_t* bytes);

/* Clear the status word and stamp the work space as prepared. Call once after allocating. */
int loop_workspace_init(void* ws, size_t ws_bytes, void* stream);

/* Residual r = -(1/T) u_s - u u_x - u_xx - u_xxxx (eq. KS_R), truncated to the band.
 * T[nloops] periods; uhat, rhat: nloops spectra in rfft layout. rhat must not alias uhat. */
int loop_residual(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat,
                  double* rhat, void* ws, size_t ws_bytes, void* stream);

/* Cost J = 1/2 int int r^2 dx ds (half of eq. cost_function), one per loop into J[nloops]. */
int loop_cost(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat,
              double* J, void* ws, size_t ws_bytes, void* stream);

/* Adjoint gradient (eq. KS_G, App. B):
 *   Ghat = G_1 = -(1/T) r_s - u r_x + r_xx + r_xxxx (band, rfft layout),
 *   dJdT[l] = int int (1/T^2) u_s r dx ds = -G_2,   J[l] as in loop_cost.
 * Any of dJdT, J may be NULL. Ghat must not alias uhat. */
int loop_adjoint_grad(double L, int Nx, int Ns, int nloops, const double* T,
                      const double* uhat, double* Ghat, double* dJdT, double* J,
                      void* ws, size_t ws_bytes, void* stream);

/* Hand-written reverse mode of J (the adjoint of Sec. 3 and App. B): the gradient of
 * sum_l gJ[l] J_l with respect to the rfft-layout coefficients and the periods, in the
 * complex convention grad = dJ/dRe + i dJ/dIm:
 *   grad_uhat = -gJ[l] w_j L G_1 in the band (w_0 = 1, w_j = 2 for j >= 1), 0 elsewhere;
 *   grad_T[l] = gJ[l] dJ/dT.
 * gJ may be NULL (all ones). Intermediates are recomputed, not stored. grad_uhat must not
 * alias uhat. */
int loop_cost_grad(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat,
                   const double* gJ, double* grad_uhat, double* grad_T, void* ws, size_t ws_bytes,
                   void* stream);

/* ---- Band layout and the reverse mode from a saved residual.
 *
 * Band layout: the retained coefficients alone, nloops x C x NB complex values with
 * C = Kx + 1 and NB = 2 Ks + 1. Element [l][j][kk] holds u_hat_{j,k} of loop l for
 * j = 0 .. Kx and kk = k (0 <= k <= Ks) or kk = k + NB (-Ks <= k < 0). As in the rfft layout,
 * an entry with j >= 1 stands for itself and its partner (-j, -k), and column j = 0 holds
 * both partners (k, -k) and is read through its Hermitian part. For the 256 x 1024 grid this
 * is 0.44 of the rfft layout's size (the modes outside the band are always zero).
 * loop_to_band / loop_from_band convert between the layouts (out of place; loop_to_band makes
 * column 0 Hermitian, loop_from_band writes 0 outside the band).
 *
 * The cost of Sec. 3 as a forward and a reverse pass, for differentiation (eq. J_variation,
 * eq. KS_L_dagger, App. B). The forward evaluates J = 1/2 int int r^2 and dJ/dT (each nloops,
 * dJdT may be NULL) and leaves the residual r_hat in `rsave` (band layout, nloops x C x NB
 * complex, caller-owned): the state-sized quantity the reverse pass needs. The reverse pass
 * forms r_x from the saved residual, needs u on the grid, and applies the adjoint operator,
 * G_1 = -(1/T) r_s - u r_x + r_xx + r_xxxx (eq. KS_G). It writes the gradient of
 * sum_l gJ[l] J_l in the complex convention dJ/dRe + i dJ/dIm, in the layout of u:
 *   grad_u = -gJ[l] w_j L G_1 in the band (w_0 = 1, w_j = 2 for j >= 1), 0 elsewhere,
 *   grad_T[l] = gJ[l] dJdT[l] (dJdT from the forward; grad_T may be NULL),
 * gJ may be NULL (all ones). The results equal loop_adjoint_grad's G_1 (scaled) bit for bit.
 * `usave` trades memory for work. NULL: the reverse pass recomputes u on the grid from u_hat
 * (one more inverse s-transform per column) and stores nothing grid-sized. Otherwise a
 * caller-owned buffer of nloops x C x Ns complex values ([l][j][n]: the x-coefficient j of u at
 * s-grid point n, i.e. the forward's inverse s-transform of each retained column) that the
 * forward fills and the reverse pass reads in place of recomputing it; pass the same buffer,
 * unchanged, to the reverse pass of the same u (the results are bitwise those without it).
 * With usave the reverse pass does not read u.
 * `layout` is LOOP_LAYOUT_RFFT or LOOP_LAYOUT_BAND for u and grad_u. rsave and usave must not
 * alias u or each other; grad_u must alias none of u, rsave, usave. Work space:
 * loop_workspace_bytes. */
typedef enum { LOOP_LAYOUT_RFFT = 0, LOOP_LAYOUT_BAND = 1 } loop_layout;
int loop_to_band(int Nx, int Ns, int nloops, const double* uhat, double* uband, void* stream);
int loop_from_band(int Nx, int Ns, int nloops, const double* uband, double* uhat, void* stream);
int loop_cost_fwd(double L, int Nx, int Ns, int nloops, int layout, const double* T, const double* u,
                  double* J, double* dJdT, double* rsave, double* usave, void* ws, size_t ws_bytes,
                  void* stream);
int loop_cost_bwd(double L, int Nx, int Ns, int nloops, int layout, const double* T, const double* u,
                  const double* rsave, const double* usave, const double* dJdT, const double* gJ,
                  double* grad_u, double* grad_T, void* ws, size_t ws_bytes, void* stream);

/* The fictitious-time update of Sec. 4.2 from the gradient of sum_l J_l (gJ = 1) in the
 * convention above, in one kernel per array: G_1 = -grad_u / (w_j L) in the band, then
 *   u <- canonical(u) + dtau * sigma_{j,k} * G_1,  sigma = 1 (EXPLICIT) or
 *   1 / (1 - dtau lambda_{j,k}(T)) (IMEX), and T <- T - dtau * grad_T,
 * with lambda and T as in loop_step (the period at the start of the step). `layout` as for
 * loop_cost_bwd; in the rfft layout every entry outside the band is set to 0. */
int loop_update_grad(double L, int Nx, int Ns, int nloops, int layout, double* T, double* u,
                     const double* grad_u, const double* grad_T, double dtau, int scheme, void* stream);

/* nsteps fictitious-time steps in place (Sec. 4.2):
 *   EXPLICIT: u_hat <- u_hat + dtau * G_1
 *   IMEX:     u_hat <- u_hat + dtau * G_1 / (1 - dtau * lambda_{j,k}(T)), the semi-implicit Euler
 *             step with the linear part lambda = -(2 pi k/T)^2 - q^8 + 2 q^6 - q^4 implicit
 *   T <- T - dtau * dJ/dT (explicit Euler), both from the state at the start of the step.
 * uhat is first made canonical in place (band-limited, real column 0). J_hist, if not NULL,
 * receives J at the start of every step as J_hist[step * nloops + l]. */
int loop_step(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau,
              int scheme, int nsteps, double* J_hist, void* ws, size_t ws_bytes, void* stream);

/* loop_step for callers that cannot allocate device memory: code recorded under HIP graph
 * capture, tight serving loops, and harnesses that forbid hipMalloc. Same arguments, steps and
 * results as loop_step (the same kernels run), but no caller work space: the work space is a
 * static device array of LOOP_NOALLOC_SCRATCH_BYTES inside the library, one per device, held
 * from the library's load until the process ends. The call allocates and frees nothing.
 * - A shape whose work space (loop_workspace_bytes(Nx, Ns, nloops)) exceeds
 *   LOOP_NOALLOC_SCRATCH_BYTES is rejected with LOOP_EWORKSPACE before anything is queued.
 * - The device must have been initialised (loop_init, or any earlier call that creates the
 *   device's twiddle table); otherwise LOOP_EINVAL.
 * - Every call on a device shares that device's array, and the array keeps the last call's
 *   contents. Each call first clears the status word it holds. Calls that overlap on one device
 *   (on different streams, or from different threads) race on the array: order them on one
 *   stream.
 * - status: if not NULL, a device int that receives the call's device status once its work
 *   has run (0, or LOOP_ENONFINITE as loop_status_sync would report it); NULL to skip. */
#define LOOP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int loop_step_noalloc(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                      int nsteps, double* J_hist, int* status, void* stream);

/* Centre-symmetric loops (Sec. 3, eq. KS_loop_sym). A loop invariant under
 * Xi: (x, s) -> (-x, s), u -> -u (u odd in x at every s) stays invariant under the flow, and
 * every field of the step then has a fixed parity in x: odd fields have purely imaginary,
 * even ones real x-spectra, column j = 0 vanishes and each column is the transform of a real
 * sequence in s. loop_step_xi takes nsteps steps storing one real number per (j, s) and the
 * k >= 0 half of the band, so state and step traffic halve, and each column transform
 * carries two columns. Input and output use loop_step's rfft layout; the input is first
 * projected orthogonally onto centre-symmetric loops (u_hat_{j,k} -> (u_hat_{j,k} -
 * conj u_hat_{j,-k}) / 2, column 0 and everything outside the band -> 0), so for an invariant
 * loop the results are loop_step's to rounding, and the output is invariant exactly.
 * Nx <= 512 (LOOP_ENOTSUP otherwise). Work space: loop_step_xi_workspace_bytes (about half of
 * loop_workspace_bytes; a loop_workspace_bytes work space also serves), prepared by
 * loop_workspace_init. Other errors, T and J_hist as loop_step; nsteps = 0 only projects. */
int loop_step_xi_workspace_bytes(int Nx, int Ns, int nloops, size_t* bytes);
int loop_step_xi(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                 int nsteps, double* J_hist, void* ws, size_t ws_bytes, void* stream);

/* The paper's own evaluation of the flow (Sec. 4.2, eq. KS_G_1), for cross-checks and for
 * the paper's step: G_1 = lambda u_hat + P(G_1NL), where
 *   G_1NL = -5 u_xxxx u_x - 10 u_xxx u_xx - 3 u_xx u_x + u^2 u_xx + u u_x^2 + (2u/T) u_xs
 *           + (1/T) u_x u_s
 * is formed pointwise on the Nx x Ns grid from derivatives taken in spectral space, and P
 * is the transform back with the two-thirds truncation. dJ/dT = int int (1/T^2) u_s r and
 * J = 1/2 int int r^2 take their integrands on the grid, with r = -(1/T) u_s - u u_x - u_xx -
 * u_xxxx formed pointwise (the paper's (0, 0)-mode rule).
 * The cubic products of G_1NL alias under the two-thirds rule and no intermediate is
 * truncated, so this G differs from loop_adjoint_grad's by aliasing and truncation errors:
 * the two agree to rounding where every product stays in the band (modes |j| <= Kx/2,
 * |k| <= Ks/2), dJ/dT agrees on every loop, and J is at least loop_cost's (the grid residual
 * keeps the out-of-band part of u u_x).
 * loop_expanded_grad: Ghat (rfft layout, band), dJdT and J (each nloops, NULL to skip), as
 * loop_adjoint_grad. loop_step_expanded: nsteps steps u_hat' = (u_hat + dtau P(G_1NL)) /
 * (1 - dtau lambda) (IMEX) or u_hat + dtau G_1 (explicit), T' = T - dtau dJ/dT; J_hist and
 * errors as loop_step. Nx <= 512 (LOOP_ENOTSUP otherwise). Work space: loop_workspace_bytes. */
int loop_expanded_grad(double L, int Nx, int Ns, int nloops, const double* T, const double* uhat, double* Ghat,
                       double* dJdT, double* J, void* ws, size_t ws_bytes, void* stream);
int loop_step_expanded(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                       int nsteps, double* J_hist, void* ws, size_t ws_bytes, void* stream);

/* Linear extrapolation of whole loops along their trajectory (App. C), in place:
 *   uhat <- uhat + factor[l] (uhat - uhat_a), T[l] <- T[l] + factor[l] (T[l] - T_a[l]),
 * for nloops loops in the rfft layout; factor (device, nloops) = 0 leaves a loop unchanged.
 * Both states should be canonical (as loop_step leaves them); then the result is too. */
int loop_extrapolate(int Nx, int Ns, int nloops, double* T, double* uhat, const double* T_a,
                     const double* uhat_a, const double* factor, void* stream);

/* Convergence driver (Sec. 4.3, App. C). Advances the loops with loop_step, `stride` steps
 * at a time, examining J of every loop on the state after each stride (and the initial one),
 * until J < J_tol for every loop or max_steps steps. With `accelerate`, each loop also
 * alternates with linear extrapolations along its trajectory: the first interval starts at
 * the first examined state with sqrt(J) <= sqrtJ_first (J = 1/2 int int r^2, half the paper's J:
 * the paper's start, sqrt(J_paper) <= 1e-3, is sqrtJ_first = 1e-3 / sqrt(2); the tests and the
 * oracle use 1e-3, i.e. sqrt(J_paper) <= sqrt(2) 1e-3); an interval ends at
 * the first examined state with sqrt(J) at most half its value at the interval's start, and
 * the loop is then replaced by l_b + rho/(1 - rho) (l_b - l_a), rho = sqrt(J_b / J_a), from the
 * interval's end states l_a, l_b; the next interval starts at the extrapolated state.
 * On return each converged loop holds the state at which it first had J < J_tol (later steps
 * of the batch do not change it), the others their last state. Host outputs (nloops each):
 * steps (the step count at convergence, or -1), extrapolations, J_final. Synchronises
 * `stream` at every examination and allocates its own device buffers (two copies of the
 * loops); a non-finite J returns LOOP_ENONFINITE. */
int loop_converge(double L, int Nx, int Ns, int nloops, double* T, double* uhat, double dtau, int scheme,
                  double J_tol, int stride, long long max_steps, int accelerate, double sqrtJ_first,
                  long long* steps, int* extrapolations, double* J_final, void* ws, size_t ws_bytes,
                  void* stream);

/* loop_step runs in one of two forms, with the same results:
 *   resident: one block per loop holds the loop's band state and intermediates in LDS and
 *     takes every step in a single launch; HBM traffic is the state's load and store. It
 *     exists where the loop's working set fits one CU's LDS (loop_resident_supported);
 *   per-pass: five kernels per step over all loops, intermediates in the work space (HBM).
 * A step of the resident form equals the per-pass form of loop_batch_step (and of loop_step
 * with nloops = 1) bit for bit; with nloops > 1 and Ns below the row-tile height the two pair
 * rows of different loops differently in the row transforms and agree to rounding.
 * loop_set_resident(mode) sets the choice for later calls in this process: 0 per-pass always,
 * 1 (default) resident where it was measured faster (for shapes whose passes take one round
 * per block, up to two loops per CU; for the others, up to one loop per CU and at least 16
 * loops), 2 resident wherever it exists.
 * It returns the previous mode, or LOOP_EINVAL for other values.
 * loop_resident_supported returns 1 when the resident form exists for an Nx x Ns loop on the
 * current device, else 0. loop_step_form returns the form loop_step takes for nloops loops of
 * Nx x Ns under the current mode: 1 resident, 0 per-pass (LOOP_EINVAL for a bad shape). */
int loop_set_resident(int mode);
int loop_resident_supported(int Nx, int Ns);
int loop_step_form(int Nx, int Ns, int nloops);

/* The update half of loop_step (the semi-implicit Euler step of Sec. 4.2), for a G_1 computed
 * elsewhere: uhat <- canonical(uhat) + dtau * sigma * Ghat (band), T <- T - dtau * dJdT[l],
 * with sigma as in loop_step. */
int loop_update(double L, int Nx, int Ns, int nloops, double* T, double* uhat,
                const double* Ghat, const double* dJdT, double dtau, int scheme, void* stream);

/* ---- Batched form: loops of uneven (L, Nx, Ns) advanced together by one persistent kernel.
 * The step is the one loop_step takes (Sec. 4.2), applied to every loop of the batch.
 *
 * loop_batch_create builds a plan on the current device. This host call allocates the
 * plan's device tables and runs a small probe kernel on the null stream (it finds the XCDs the
 * persistent schedule uses) and waits for it, so it must run outside stream capture. Each loop needs a power-of-
 * two Nx in [8, 512] and Ns in [8, 1024]. The loops' spectra live back to back in one
 * rfft-layout pool, in the order given, at the offsets loop_batch_info reports (in complex
 * values). Periods T[nloops]; J_hist, if not NULL, is [nsteps][nloops].
 *
 * loop_batch_step queues its kernels on `stream`, and allocates and synchronises nothing:
 * a conversion into band layout (which also makes every loop canonical), the steps (see
 * loop_batch_set_schedule), and the conversion back. Its work space
 * (loop_batch_info bytes) must be prepared once by loop_batch_workspace_init; a call that
 * ended in LOOP_EHANG leaves it ready for the next call. */
typedef enum { LOOP_BATCH_PER_PASS = 0, LOOP_BATCH_PERSISTENT = 1, LOOP_BATCH_STREAMS = 2 } loop_batch_schedule;
int loop_batch_create(int nloops, const double* L, const int* Nx, const int* Ns, void** plan);
/* Choose how loop_batch_step runs the steps (results are identical bit for bit):
 *   LOOP_BATCH_PER_PASS (default): one kernel per pass over every loop's tiles, four per step;
 *   LOOP_BATCH_PERSISTENT: one launch for all steps. Each loop is assigned to one XCD, and
 *   blocks pull (pass, loop, tile) items of their own XCD's list in dependency order, so that
 *   every hand-over between blocks stays within one L2 (see the scheduler notes in the
 *   source). loop_batch_create finds the XCDs with a probe launch; a block on an XCD the
 *   probe did not see leaves and sets LOOP_ENOTSUP. It measured 1.5-2.5x slower than the
 *   other two, and
 *   loop_batch_autotune does not choose it;
 *   LOOP_BATCH_STREAMS: the loops split into K groups of about equal work (K from
 *   loop_batch_set_streams, 2 to 4, default 2), group 0 on `stream` and the others on streams
 *   the plan owns (default priority), each started one pass after the previous group, so that
 *   different passes of different groups run side by side as separate kernels. The plan's
 *   streams are forked from and joined back to `stream` with events, so the call stays
 *   ordered on `stream` and can be captured in a graph from it. Calls with one plan must not
 *   overlap (the plan's streams and events are shared). */
int loop_batch_set_schedule(void* plan, int schedule);
int loop_batch_set_streams(void* plan, int nstreams);
/* Bound, in seconds, of one dependency wait of the persistent schedule (default 2; 0 to 3600).
 * A wait that runs out abandons the launch: every block leaves at its next wait, the status
 * word becomes LOOP_EHANG, and the state the call leaves behind is not a step. The counters
 * the schedule uses are cleared before each launch, so the next call runs normally. */
int loop_batch_set_wait_limit(void* plan, double seconds);
int loop_batch_destroy(void* plan);
int loop_batch_info(const void* plan, size_t* ws_bytes, size_t* pool_elems, long long* uhat_offsets);
int loop_batch_workspace_init(const void* plan, void* ws, size_t ws_bytes, void* stream);
int loop_batch_step(const void* plan, double* T, double* uhat_pool, double dtau, int scheme,
                    int nsteps, double* J_hist, void* ws, size_t ws_bytes, void* stream);

/* The building blocks of loop_batch_step's per-pass schedule, for callers that interleave
 * other work or time each kernel. Run loop_batch_load, then pass 0 (A) once, then passes
 * 1..4 (B, C, D, E) for step = 0 .. nsteps-1, then loop_batch_store. This equals
 * loop_batch_step(..., nsteps, ...) bit for bit. The pass numbering:
 *   0 A: inverse s-transforms of the band columns;
 *   1 B: rows, u * u_x;
 *   2 C: columns, residual (eq. KS_R), partial J and dJ/dT, linear part of the flow;
 *   3 D: rows, u * r_x, J and dJ/dT, period update;
 *   4 E: columns, G_1 (eq. KS_G) and the state update, plus the next step's A unless step
 *        is the last. */
int loop_batch_load(const void* plan, const double* uhat_pool, void* ws, size_t ws_bytes, void* stream);
int loop_batch_pass(const void* plan, int pass, int step, int nsteps, double* T, double dtau, int scheme,
                    double* J_hist, void* ws, size_t ws_bytes, void* stream);
int loop_batch_store(const void* plan, double* uhat_pool, void* ws, size_t ws_bytes, void* stream);

/* Kernel variants and the autotuner (per-pass schedule). Each pass has up to
 * LOOP_BATCH_VARIANTS kernel variants. They differ in the range of transform sizes compiled
 * in (hence register use and wavefronts per SIMD) and, for the row passes B and D, in how
 * tiles of rows reach LDS and in the FFT tile shape:
 *   row passes:    0 sizes 8..512 staged through registers; 1 sizes 8..64 staged;
 *                  2 sizes 8..64 copied by the load unit straight into LDS;
 *                  3 sizes 8..64 staged, 4 points per thread (8 elsewhere): twice the
 *                    threads per row transform, half-height tiles;
 *   column passes: 0 sizes 8..1024; 1 sizes 8..64; 2 sizes 8..512.
 * Variants 0-2 of a pass run the same arithmetic, so they agree bit for bit. Row variant 3
 * pairs rows and factors the transforms differently and agrees to rounding (it meets the
 * same 1e-12 per-step bound against the definitions).
 * A variant is usable for a plan when its size range covers every loop's Nx (row passes)
 * or Ns (column passes). A new plan takes the narrowest staged variant for every pass, or
 * the configuration an earlier loop_batch_autotune chose for a plan with the same multiset
 * of (Nx, Ns) on the same device in this process.
 *
 * loop_batch_set_variant: pass 0..4, variant 0..LOOP_BATCH_VARIANTS-1; LOOP_EINVAL when the
 * variant does not cover the plan's sizes.
 * loop_batch_get_config: any output pointer may be NULL; variants receives 5 ints, nstreams
 * the stream count of the multi-stream schedule.
 *
 * loop_batch_autotune times, on the caller's state (T[nloops], uhat_pool as for
 * loop_batch_step; neither is modified), every usable variant of every pass over `reps`
 * back-to-back launches (best of three trials, hipEvent timing on `stream`), keeps the
 * fastest per pass (the plan's current variant unless another is faster by more than 1%),
 * then times `reps` whole steps of the per-pass schedule and of the multi-stream one with 2, 3
 * and 4 streams, and keeps the fastest (the persistent schedule is not timed; its entry in the
 * report is -1). The work of every kernel is independent of dtau
 * and scheme, so the timing runs use a step of 1e-30 (IMEX), which leaves the state unchanged
 * to the last bit in practice and keeps every repetition finite. It allocates temporary
 * device copies of T and the pool, synchronises `stream`, and overwrites the work space's
 * intermediates (the work space stays prepared). reps in [1, 1000]. report, if not NULL,
 * receives 5 * LOOP_BATCH_VARIANTS + 5 doubles: the mean microseconds per launch of (pass,
 * variant) at index pass * LOOP_BATCH_VARIANTS + variant (-1 for variants not usable), then
 * microseconds per step of the per-pass, the persistent (-1, not timed), and the
 * multi-stream schedule with 2, 3 and 4 streams. Returns a device status raised while timing, else LOOP_OK. */
#define LOOP_BATCH_VARIANTS 4
int loop_batch_set_variant(void* plan, int pass, int variant);
int loop_batch_get_config(const void* plan, int* schedule, int* variants, int* nstreams);
int loop_batch_autotune(void* plan, const double* T, const double* uhat_pool, int reps, double* report, void* ws,
                        size_t ws_bytes, void* stream);

/* Kernel timing. Between loop_trace_start and loop_trace_stop, every pass kernel the library
 * queues (and the conversions, finalize and update kernels) is launched with two HIP events
 * that its own dispatch records at the kernel's start and end (hipExtLaunchKernelGGL), so a
 * duration is the kernel's alone, as a profiler's kernel trace measures it. loop_trace_stop
 * ends recording, waits for the recorded events and sums the durations per kernel; loop_trace_count and loop_trace_get
 * then report, per kernel name (as in "k_rowD<256>" or "k_rag<3, 1>", in order of first
 * launch): launches, total, shortest and longest duration in microseconds. Host calls that
 * create events: not for use under stream capture. loop_trace_stop returns LOOP_EHIP if an
 * event could not be created, recorded or read (the counts then cover the rest). */
int loop_trace_start(void);
int loop_trace_stop(void);
int loop_trace_count(void);
int loop_trace_get(int i, char* name, int name_len, long long* launches, double* total_us, double* min_us,
                   double* max_us);

/* Read (and clear) the sticky device status of a work space. Waits for `stream`. */
int loop_status_sync(void* ws, void* stream);

/* Human-readable text for a loop_status value. */
const char* loop_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* LOOPORBIT_H */
