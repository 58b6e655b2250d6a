"""Initial loops from chaotic Kuramoto-Sivashinsky runs (Sec. 4.3).

TEST INFRASTRUCTURE. The parity reference for the device pipeline that turns a chaotic KS
run into initial loops; only the test suite, the stored-fixture script and the CPU-baseline
leg of the benchmark use it. It shares no code with the HIP library.

The pipeline of Sec. 4.3:

1. Integrate the KS equation u_t = -u u_x - u_xx - u_xxxx on [0, L) (eq. KS), optionally in
   the centre-symmetric subspace u(-x) = -u(x) (eq. KS_sym).
2. Record the norm ||u||(t) = sqrt(int_0^L u^2 dx) (eq. conventinal_L2norm) along the run.
3. Take pairs of maxima of ||u||(t) at times t_a < t_b with ||u||(t_b) close to ||u||(t_a);
   the segment of the run between them is a candidate with period T = t_b - t_a.
4. Fourier-transform the segment in time, drop the high temporal frequencies, and read the
   result as the field of a loop on s = (t - t_a) / T, with that period.

The paper names no integrator, no tolerances and no filter; the readings taken here:

* Integrator: ETDRK4 (Cox & Matthews, J. Comput. Phys. 176, 2002) on the Fourier-Galerkin
  system with the two-thirds rule in x, u_hat' = c u_hat + N_hat(u_hat), c_j = q_j^2 - q_j^4,
  N_hat = -(i q_j / 2) FFT(u^2) in the band. Its coefficients are evaluated here in 50-digit
  arithmetic (mpmath) from their closed forms. In the centre-symmetric subspace the state
  is projected onto odd fields (Re u_hat_j = 0, u_hat_0 = 0) after every step, so that
  rounding cannot carry the run out of the subspace.
* Samples: the state before step i * sample_every, i = 0 .. nsteps / sample_every - 1.
* Maxima: sample i with n_{i-1} < n_i >= n_{i+1}. Pairs: every pair of maxima a < b with
  Tmin <= (b - a) dt_s <= Tmax and |n_b - n_a| <= rel_tol n_a, ordered by (a, b).
* Low-pass: the n = b - a samples a .. b - 1 are one period of a time-periodic field on
  s_i = i / n; its temporal modes |k| <= kc are kept (requires n > 2 kc), the rest dropped,
  and the result, truncated to the loop's band in x, is the loop's spectrum on the loop grid.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np

# --------------------------------------------------------------------------------------------
# Fourier-Galerkin KS system (eq. KS, Sec. 4.2): rfft layout, forward-normalised
# --------------------------------------------------------------------------------------------


def band_limit(Nx: int) -> int:
    return (Nx - 1) // 3


def wavenumbers(L: float, Nx: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(Nx // 2 + 1) / L


def linear_rates(L: float, Nx: int) -> np.ndarray:
    """c_j of u_hat_j' = c_j u_hat_j + ...: -u_xx - u_xxxx -> (q^2 - q^4) u_hat."""
    q = wavenumbers(L, Nx)
    return q * q - q ** 4


def truncate(vhat: np.ndarray) -> np.ndarray:
    Nx = 2 * (vhat.shape[-1] - 1)
    out = np.array(vhat, dtype=np.complex128, copy=True)
    out[..., band_limit(Nx) + 1:] = 0.0
    return out


def to_grid(vhat: np.ndarray) -> np.ndarray:
    Nx = 2 * (vhat.shape[-1] - 1)
    return np.fft.irfft(vhat, n=Nx, norm="forward")


def from_grid(v: np.ndarray) -> np.ndarray:
    return np.fft.rfft(v, norm="forward")


def nonlinear(uhat: np.ndarray, L: float) -> np.ndarray:
    """-u u_x = -(u^2)_x / 2 in the band: the grid square of the band-limited field, its
    transform, the derivative i q_j and the two-thirds truncation."""
    Nx = 2 * (uhat.shape[-1] - 1)
    u = to_grid(truncate(uhat))
    return truncate(-0.5j * wavenumbers(L, Nx) * from_grid(u * u))


def symmetric_part(uhat: np.ndarray) -> np.ndarray:
    """Projection onto odd fields (eq. KS_sym): u(x) -> (u(x) - u(-x)) / 2 keeps i Im u_hat_j."""
    return 1j * np.imag(truncate(uhat))


def norm(uhat: np.ndarray, L: float) -> float:
    """||u|| = sqrt(int_0^L u^2 dx) (eq. conventinal_L2norm), by Parseval on the rfft layout."""
    w = np.full(uhat.shape[-1], 2.0)
    w[0] = 1.0
    return math.sqrt(L * float(np.sum(w * np.abs(uhat) ** 2)))


# --------------------------------------------------------------------------------------------
# ETDRK4 (Cox & Matthews 2002)
# --------------------------------------------------------------------------------------------


def etdrk4_coefficients(L: float, Nx: int, h: float):
    """Per mode, with z = h c_j: E = e^z, E2 = e^{z/2}, Q = (e^{z/2} - 1) / c and
        f1 = h (-4 - z + e^z (4 - 3z + z^2)) / z^3,
        f2 = h (2 + z + e^z (-2 + z)) / z^3,
        f3 = h (-4 - 3z - z^2 + e^z (4 - z)) / z^3,
    with their limits h/2, h/6, h/6, h/6 at z = 0. Evaluated with 50 significant digits."""
    mpmath.mp.dps = 50
    out = {k: np.zeros(Nx // 2 + 1) for k in ("E", "E2", "Q", "f1", "f2", "f3")}
    for j, c in enumerate(linear_rates(L, Nx)):
        cm = mpmath.mpf(float(c))
        hm = mpmath.mpf(h)
        z = hm * cm
        if z == 0:
            vals = (1, 1, hm / 2, hm / 6, hm / 6, hm / 6)
        else:
            ez = mpmath.exp(z)
            vals = (ez, mpmath.exp(z / 2), (mpmath.exp(z / 2) - 1) / cm,
                    hm * (-4 - z + ez * (4 - 3 * z + z * z)) / z ** 3,
                    hm * (2 + z + ez * (-2 + z)) / z ** 3,
                    hm * (-4 - 3 * z - z * z + ez * (4 - z)) / z ** 3)
        for key, v in zip(("E", "E2", "Q", "f1", "f2", "f3"), vals):
            out[key][j] = float(v)
    return out


def etdrk4_step(uhat: np.ndarray, L: float, co: dict) -> np.ndarray:
    """One ETDRK4 step:
        a = E2 u + Q N(u),  b = E2 u + Q N(a),  c = E2 a + Q (2 N(b) - N(u)),
        u' = E u + f1 N(u) + 2 f2 (N(a) + N(b)) + f3 N(c)."""
    Nu = nonlinear(uhat, L)
    a = co["E2"] * uhat + co["Q"] * Nu
    Na = nonlinear(a, L)
    b = co["E2"] * uhat + co["Q"] * Na
    Nb = nonlinear(b, L)
    c = co["E2"] * a + co["Q"] * (2.0 * Nb - Nu)
    Nc = nonlinear(c, L)
    return truncate(co["E"] * uhat + co["f1"] * Nu + 2.0 * co["f2"] * (Na + Nb) + co["f3"] * Nc)


def integrate(uhat: np.ndarray, L: float, dt: float, nsteps: int, sample_every: int = 1,
              symmetric: bool = False):
    """nsteps ETDRK4 steps of one run. Returns (final state, norms, snapshots): the samples
    are the states before steps 0, s, 2s, ... (s = sample_every, nsteps a multiple of s)."""
    if nsteps % sample_every:
        raise ValueError("nsteps must be a multiple of sample_every")
    Nx = 2 * (uhat.shape[-1] - 1)
    co = etdrk4_coefficients(L, Nx, dt)
    u = symmetric_part(uhat) if symmetric else truncate(uhat)
    ns = nsteps // sample_every
    norms = np.zeros(ns)
    snaps = np.zeros((ns, Nx // 2 + 1), dtype=np.complex128)
    for i in range(nsteps):
        if i % sample_every == 0:
            norms[i // sample_every] = norm(u, L)
            snaps[i // sample_every] = u
        u = etdrk4_step(u, L, co)
        if symmetric:
            u = symmetric_part(u)
    return u, norms, snaps


# --------------------------------------------------------------------------------------------
# recurrences of ||u||(t) and the temporal low-pass (Sec. 4.3)
# --------------------------------------------------------------------------------------------


def maxima(norms) -> list:
    """Samples i with n_{i-1} < n_i >= n_{i+1}."""
    return [i for i in range(1, len(norms) - 1) if norms[i - 1] < norms[i] >= norms[i + 1]]


def recurrences(norms, dt_s: float, rel_tol: float, Tmin: float, Tmax: float) -> list:
    """Pairs (a, b) of maxima with Tmin <= (b - a) dt_s <= Tmax and |n_b - n_a| <= rel_tol n_a,
    in increasing (a, b)."""
    m = maxima(norms)
    out = []
    for p, a in enumerate(m):
        for b in m[p + 1:]:
            T = (b - a) * dt_s
            if T > Tmax:
                break
            if T >= Tmin and abs(norms[b] - norms[a]) <= rel_tol * norms[a]:
                out.append((a, b))
    return out


def segment_to_loop(snaps: np.ndarray, a: int, b: int, dt_s: float, Ns: int, kc: int):
    """The loop of the segment of samples a .. b - 1: its temporal transform over one period
    (n = b - a samples on s_i = i / n), modes |k| <= kc kept, on the (Ns, Nx) loop grid in
    the rfft layout of the loop oracle. Returns (u_hat, T)."""
    n = b - a
    if n <= 2 * kc or kc > (Ns - 1) // 3:
        raise ValueError("need n > 2 kc and kc within the loop band")
    seg = snaps[a:b]  # (n, Nx/2+1): u_hat_j(t_a + i dt_s)
    H = seg.shape[1]
    Nx = 2 * (H - 1)
    ck = np.fft.fft(seg, axis=0) / n  # c_{j,k} = (1/n) sum_i u_hat_j(t_i) e^{-2 pi i k i / n}
    out = np.zeros((Ns, H), dtype=np.complex128)
    for k in range(-kc, kc + 1):
        out[k % Ns, :] = ck[k % n, :]
    out[:, band_limit(Nx) + 1:] = 0.0
    return out, n * dt_s
