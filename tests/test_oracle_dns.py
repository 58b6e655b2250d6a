"""Pins of the initial-loop oracle (oracle/ks_dns.py, Sec. 4.3) against what the mathematics
fixes: the integral form of the ETDRK4 coefficients, exact exponential evolution where the
nonlinear term vanishes, a library ODE integrator, fourth-order convergence, the nonlinear
term by direct convolution, its energy neutrality, the invariance of the odd subspace,
Parseval, brute-force recurrence search and closed-form segments."""
import math

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

import loopgen
from oracle import ks_dns as D


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ---------------------------------------------------------------- ETDRK4 coefficients
def phi(k, z):
    """phi_k(z) = int_0^1 exp((1 - t) z) t^(k-1) / (k-1)! dt, by adaptive quadrature."""
    return quad(lambda t: math.exp((1.0 - t) * z) * t ** (k - 1) / math.factorial(k - 1), 0.0, 1.0,
                epsabs=0.0, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("L,Nx,h", [(39.0, 64, 0.05), (22.0, 32, 0.25), (100.0, 128, 0.01)])
def test_coefficients_match_their_integral_form(L, Nx, h):
    co = D.etdrk4_coefficients(L, Nx, h)
    c = D.linear_rates(L, Nx)
    for j in range(0, Nx // 2 + 1, 3):
        z = h * c[j]
        assert abs(co["E"][j] - math.exp(z)) <= 1e-15 * math.exp(z)
        assert abs(co["E2"][j] - math.exp(z / 2)) <= 1e-15 * math.exp(z / 2)
        p1, p2, p3 = phi(1, z), phi(2, z), phi(3, z)
        assert abs(co["Q"][j] - 0.5 * h * phi(1, z / 2)) <= 1e-12 * abs(co["Q"][j])
        assert abs(co["f1"][j] - h * (p1 - 3 * p2 + 4 * p3)) <= 1e-11 * h
        assert abs(co["f2"][j] - h * (p2 - 2 * p3)) <= 1e-11 * h
        assert abs(co["f3"][j] - h * (-p2 + 4 * p3)) <= 1e-11 * h


def test_coefficients_reduce_to_rk4_weights_without_linear_part():
    co = D.etdrk4_coefficients(39.0, 64, 0.1)
    assert co["E"][0] == 1.0 and co["Q"][0] == 0.05
    assert co["f1"][0] == co["f2"][0] == co["f3"][0] == 0.1 / 6


# ---------------------------------------------------------------- the Galerkin system
def brute_nonlinear(uhat, L):
    """-(i q_j / 2) sum_{j1 + j2 = j} u_{j1} u_{j2} over the band, u_{-j} = conj u_j."""
    Nx = 2 * (len(uhat) - 1)
    K = (Nx - 1) // 3
    full = {j: (uhat[j] if j >= 0 else np.conj(uhat[-j])) for j in range(-K, K + 1)}
    out = np.zeros_like(uhat)
    for j in range(0, K + 1):
        s = sum(full[j1] * full[j - j1] for j1 in range(-K, K + 1) if -K <= j - j1 <= K)
        out[j] = -0.5j * (2 * math.pi * j / L) * s
    return out


@pytest.mark.parametrize("Nx", [8, 16, 32])
def test_nonlinear_term_is_the_band_convolution(Nx):
    rng = np.random.default_rng(Nx)
    u = loopgen.random_ks_state(rng, Nx)
    u[0] = 0.7  # a mean mode as well
    assert rel(D.nonlinear(u, 13.0), brute_nonlinear(u, 13.0)) < 1e-14


def test_nonlinear_term_conserves_energy():
    rng = np.random.default_rng(3)
    for Nx in (16, 64, 256):
        u = loopgen.random_ks_state(rng, Nx)
        N = D.nonlinear(u, 39.0)
        w = np.full(len(u), 2.0)
        w[0] = 1.0
        assert abs(np.sum(w * np.real(np.conj(u) * N))) < 1e-14 * np.sum(w * np.abs(u) * np.abs(N))


def test_norm_is_the_grid_integral():
    rng = np.random.default_rng(4)
    L, Nx = 39.0, 64
    u = loopgen.random_ks_state(rng, Nx)
    x = D.to_grid(u)
    assert abs(D.norm(u, L) - math.sqrt(np.sum(x * x) * L / Nx)) < 1e-14 * D.norm(u, L)


def test_single_out_of_band_mode_evolves_exactly():
    """u = A e^{i q_j x} + c.c. with 2j beyond the band: u^2 has modes 0 and 2j only, so N = 0
    and the exact solution is u_hat_j(t) = e^{c_j t} u_hat_j(0)."""
    L, Nx, h = 39.0, 64, 0.05
    K = (Nx - 1) // 3
    for j in (K // 2 + 1, K):
        u0 = np.zeros(Nx // 2 + 1, dtype=np.complex128)
        u0[j] = 0.3 - 0.2j
        u, _, _ = D.integrate(u0, L, h, 40)
        c = (2 * math.pi * j / L) ** 2 - (2 * math.pi * j / L) ** 4
        assert abs(u[j] - math.exp(c * 40 * h) * u0[j]) <= 1e-13 * abs(u0[j])
        assert np.max(np.abs(np.delete(u, j))) <= 1e-15 * abs(u0[j])  # rounding of the zero product


def galerkin_rhs(L, Nx):
    c = D.linear_rates(L, Nx)
    K = (Nx - 1) // 3

    def f(t, y):
        u = np.zeros(Nx // 2 + 1, dtype=np.complex128)
        u[:K + 1] = y[:K + 1] + 1j * y[K + 1:]
        du = c * u + brute_nonlinear(u, L)
        return np.concatenate([du[:K + 1].real, du[:K + 1].imag])
    return f, K


def test_matches_a_library_integrator_to_fourth_order():
    """Against scipy's DOP853 at tight tolerance on the same Galerkin system (right-hand side
    by direct convolution): the error is O(h^4) and halves the step -> / 16."""
    L, Nx, tend = 22.0, 16, 2.0
    rng = np.random.default_rng(5)
    u0 = loopgen.random_ks_state(rng, Nx, scale=0.5)
    f, K = galerkin_rhs(L, Nx)
    sol = solve_ivp(f, (0.0, tend), np.concatenate([u0[:K + 1].real, u0[:K + 1].imag]), method="DOP853",
                    rtol=1e-13, atol=1e-15)
    ref = sol.y[:K + 1, -1] + 1j * sol.y[K + 1:, -1]
    errs = []
    for n in (20, 40, 80):
        u, _, _ = D.integrate(u0, L, tend / n, n)
        errs.append(np.max(np.abs(u[:K + 1] - ref)))
    assert errs[-1] < 1e-8
    for e1, e2 in zip(errs, errs[1:]):
        assert 11.0 < e1 / e2 < 22.0, errs


def test_odd_fields_stay_odd():
    L, Nx = 39.0, 64
    rng = np.random.default_rng(6)
    u0 = loopgen.random_ks_state(rng, Nx, scale=0.5, odd=True)
    u, _, _ = D.integrate(u0, L, 0.05, 200)
    assert np.max(np.abs(u.real)) < 1e-13 * np.max(np.abs(u))
    us, _, _ = D.integrate(u0, L, 0.05, 200, symmetric=True)
    assert rel(us, u) < 1e-12
    assert np.all(us.real == 0)


def test_samples_are_the_states_before_their_steps():
    L, Nx = 39.0, 32
    u0 = loopgen.random_ks_state(np.random.default_rng(7), Nx, scale=0.3)
    u, n, s = D.integrate(u0, L, 0.05, 12, sample_every=4)
    assert len(n) == 3 and np.array_equal(s[0], D.truncate(u0))
    u4, _, _ = D.integrate(u0, L, 0.05, 4)
    assert np.array_equal(s[1], u4)
    assert n[1] == D.norm(u4, L)
    u8, _, _ = D.integrate(u4, L, 0.05, 4)
    u12, _, _ = D.integrate(u8, L, 0.05, 4)
    assert np.array_equal(s[2], u8) and np.array_equal(u, u12)
    with pytest.raises(ValueError):
        D.integrate(u0, L, 0.05, 10, sample_every=4)


# ---------------------------------------------------------------- recurrences
def brute_recurrences(n, dt_s, tol, Tmin, Tmax):
    idx = range(1, len(n) - 1)
    mx = {i for i in idx if n[i - 1] < n[i] and n[i] >= n[i + 1]}
    return sorted((a, b) for a in mx for b in mx
                  if a < b and Tmin <= (b - a) * dt_s <= Tmax and abs(n[b] - n[a]) <= tol * n[a])


def test_maxima_of_a_known_series():
    t = np.arange(400) * 0.1
    n = 2.0 + np.sin(2 * np.pi * t / 5.0 + 0.3)  # maxima where the phase is pi/2 (mod 2 pi)
    m = D.maxima(n)
    expect = [int(round((np.pi / 2 - 0.3 + 2 * np.pi * q) / (2 * np.pi) * 50)) for q in range(8)]
    assert m == expect
    # a plateau of equal values counts once, at its first sample
    assert D.maxima(np.array([0.0, 1.0, 1.0, 1.0, 0.0])) == [1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_recurrences_equal_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = np.round(rng.uniform(1.0, 2.0, size=600), 2)  # ties included
    got = D.recurrences(n, 0.1, 0.02, 2.0, 9.0)
    assert got == brute_recurrences(n, 0.1, 0.02, 2.0, 9.0)
    assert len(got) > 50


# ---------------------------------------------------------------- segments to loops
def test_travelling_wave_segment_is_one_loop_mode():
    """u(x, t) = A sin(q_1 (x - c t)) over exactly one period P = n dt_s: u_hat_1(t) =
    (A / 2i) e^{-i q_1 c t}, i.e. the loop mode (j, k) = (1, -1) = A / 2i, with T = P."""
    L, Nx, Ns, n, dt_s, A = 39.0, 32, 32, 50, 0.2, 0.8
    q1 = 2 * math.pi / L
    c = L / (n * dt_s)
    snaps = np.zeros((n + 7, Nx // 2 + 1), dtype=np.complex128)
    for i in range(n + 7):
        snaps[i, 1] = A / 2j * np.exp(-1j * q1 * c * (i - 3) * dt_s)
    u, T = D.segment_to_loop(snaps, 3, 3 + n, dt_s, Ns, kc=5)
    expect = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    expect[-1, 1] = A / 2j
    assert abs(T - n * dt_s) < 1e-15 and np.max(np.abs(u - expect)) < 1e-15


def test_low_pass_drops_high_temporal_modes():
    Nx, Ns, n, dt_s = 16, 32, 40, 0.1
    i = np.arange(n)[:, None]
    coeff = {0: 0.5, 2: 0.25 - 0.1j, -3: 0.2j, 7: 0.3, -9: 0.1}
    snaps = np.zeros((n, Nx // 2 + 1), dtype=np.complex128)
    for k, v in coeff.items():
        snaps[:, 2:3] += v * np.exp(2j * np.pi * k * i / n)
    snaps[:, 7] = 1.0  # outside the x band of Nx = 16 (Kx = 5)
    u, T = D.segment_to_loop(snaps, 0, n, dt_s, Ns, kc=5)
    for k in range(-Ns // 2, Ns // 2):
        want = coeff.get(k, 0.0) if abs(k) <= 5 else 0.0
        assert abs(u[k % Ns, 2] - want) < 1e-15
    assert np.all(u[:, 6:] == 0) and abs(T - 4.0) < 1e-15
    with pytest.raises(ValueError):
        D.segment_to_loop(snaps, 0, 10, dt_s, Ns, kc=5)
    with pytest.raises(ValueError):
        D.segment_to_loop(snaps, 0, n, dt_s, Ns, kc=11)


def test_segments_of_odd_runs_give_centre_symmetric_loops():
    """Odd snapshots give loops invariant under Xi: u_hat_{j,k} = -conj u_hat_{j,-k}."""
    L, Nx = 39.0, 64
    u0 = loopgen.random_ks_state(np.random.default_rng(8), Nx, scale=0.5, odd=True)
    _, n, s = D.integrate(u0, L, 0.05, 400, 2, symmetric=True)
    u, T = D.segment_to_loop(s, 10, 150, 0.1, 64, kc=12)
    kneg = (-np.arange(64)) % 64
    assert np.max(np.abs(u + np.conj(u[kneg, :]))) < 1e-15 * np.max(np.abs(u))
