"""Pins for the CPU oracle: each check is fixed by the paper's equations or by mathematics,
not by re-running the oracle's own formulas.

Paper: Azimi, Ashtari & Schneider, arXiv:2007.06427.
- Brute force: explicit DFT sums and direct convolution on tiny grids (Sec. 4.2).
- Closed forms: a single travelling mode, derived by hand from eqs. KS_R, KS_L_dagger and
  KS_G.
- The adjoint identity (eq. adjoint_definition) and the directional derivative's defining
  limit (eq. directional_derivative).
- Central finite differences of J against the flow (eq. J_variation).
- Shift and Xi equivariance (Sec. 3 and eq. KS_loop_sym), descent (eq. J_variation), the
  linear limit (lambda of Sec. 4.2) and fixed points.
"""
import numpy as np
import pytest

import loopgen
from oracle import brute as B
from oracle import ks_loop as K

RNG_SEED = 12345


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)


def l2(vhat, L):
    return K.inner(vhat, vhat, L)


# ------------------------------------------------------------------------------ pi1 brute force
@pytest.mark.parametrize("Nx,Ns", [(8, 8), (12, 8), (16, 12), (8, 16)])
def test_brute_force_matches_transform_oracle(Nx, Ns):
    rng = np.random.default_rng(RNG_SEED + Nx * 100 + Ns)
    u = loopgen.random_band_field(rng, Nx, Ns)
    # out-of-band garbage and a non-Hermitian column 0 must be ignored the same way by both
    junk = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    u = u + 0.3 * junk * (~K.band_mask(Nx, Ns))
    u[1, 0] += 0.2 + 0.1j
    T, L = 17.3, 9.7
    rb, Jb, dTb, Gb = B.all_quantities(u, T, L)
    r = K.residual(u, T, L)
    G, dT, J = K.adjoint_grad(u, T, L)
    assert rel(r, rb) < 1e-13
    assert abs(J - Jb) <= 1e-13 * abs(Jb)
    assert abs(K.cost(u, T, L) - Jb) <= 1e-13 * abs(Jb)
    assert abs(dT - dTb) <= 1e-13 * abs(dTb)
    assert abs(K.dJdT(u, T, L) - dTb) <= 1e-13 * abs(dTb)
    assert rel(G, Gb) < 1e-13


def test_brute_force_grid_values_match_inverse_transform():
    rng = np.random.default_rng(RNG_SEED)
    u = loopgen.random_band_field(rng, 8, 12)
    g = B.grid_values(B.from_rfft(u), 8, 12)
    assert np.max(np.abs(g.imag)) < 1e-13
    assert rel(g.real, K.to_grid(K.canonical(u))) < 1e-14


# ------------------------------------------------------------------------------ pi2 closed form
def single_mode_case(j0, k0, A=0.7, T=13.0, L=11.0, Nx=32, Ns=32):
    """u = A cos(q x + w s) with q = 2 pi j0 / L, w = 2 pi k0.

    By hand from eq. KS_R:
        r = a sin t + b cos t + c sin 2t,  a = A w / T,  b = A (q^2 - q^4),  c = A^2 q / 2.
    From eq. KS_G, with u r_x = A q [a/2 + a/2 cos 2t - b/2 sin 2t + c cos t + c cos 3t]:
        G1 = C0 + Cc1 cos t + Cs1 sin t + Cc2 cos 2t + Cs2 sin 2t + Cc3 cos 3t.
    """
    q = 2 * np.pi * j0 / L
    w = 2 * np.pi * k0
    a, b, c = A * w / T, A * (q ** 2 - q ** 4), A * A * q / 2
    C0 = -A * q * a / 2
    Cc1 = -(w / T) * a - A * q * c + (q ** 4 - q ** 2) * b
    Cs1 = (w / T) * b + (q ** 4 - q ** 2) * a
    Cc2 = -2 * (w / T) * c - A * q * a / 2
    Cs2 = A * q * b / 2 + (16 * q ** 4 - 4 * q ** 2) * c
    Cc3 = -A * q * c
    uhat = loopgen.from_modes(Nx, Ns, [(j0, k0, A / 2)])
    r_expect = loopgen.from_modes(Nx, Ns, [(j0, k0, b / 2 - 0.5j * a), (2 * j0, 2 * k0, -0.5j * c)])
    G_expect = loopgen.from_modes(Nx, Ns, [(0, 0, 0.0)])
    G_expect[0, 0] = C0
    for (m, cc, cs) in [(1, Cc1, Cs1), (2, Cc2, Cs2), (3, Cc3, 0.0)]:
        extra = loopgen.from_modes(Nx, Ns, [(m * j0, m * k0, cc / 2 - 0.5j * cs)])
        G_expect = G_expect + extra
    J_expect = (L / 4) * (A ** 2 * w ** 2 / T ** 2 + A ** 2 * (q ** 2 - q ** 4) ** 2 + A ** 4 * q ** 2 / 4)
    dT_expect = -L * A ** 2 * w ** 2 / (2 * T ** 3)
    return uhat, T, L, r_expect, G_expect, J_expect, dT_expect


@pytest.mark.parametrize("j0,k0", [(2, 3), (1, 1), (3, 2), (0, 3), (2, 0)])
def test_single_mode_closed_form(j0, k0):
    uhat, T, L, r_e, G_e, J_e, dT_e = single_mode_case(j0, k0)
    r = K.residual(uhat, T, L)
    G, dT, J = K.adjoint_grad(uhat, T, L)
    scale = max(np.abs(r_e).max(), 1.0)
    assert np.abs(r - r_e).max() < 1e-13 * scale
    assert abs(J - J_e) <= 1e-13 * J_e
    assert abs(dT - dT_e) <= 1e-13 * max(abs(dT_e), J_e)
    assert np.abs(G - G_e).max() < 1e-12 * max(np.abs(G_e).max(), 1.0)


def test_single_mode_mean_drift_nonzero():
    """The flow has a mean-mode component -A^2 q w / (2T) for a travelling wave: no projection."""
    uhat, T, L, _, G_e, _, _ = single_mode_case(2, 3)
    G, _, _ = K.adjoint_grad(uhat, T, L)
    assert abs(G[0, 0].real - G_e[0, 0].real) < 1e-12 * abs(G_e[0, 0].real)
    assert abs(G[0, 0]) > 1e-3


# ------------------------------------------------------------------------------ pi3 adjoint identity
@pytest.mark.parametrize("Nx,Ns,L", [(16, 16, 7.0), (32, 64, 22.0), (64, 32, 39.0)])
def test_adjoint_identity(Nx, Ns, L):
    rng = np.random.default_rng(RNG_SEED + Nx + Ns)
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=min(6, (Nx - 1) // 3), kmax=min(6, (Ns - 1) // 3), scale=0.5)
    v1 = loopgen.random_band_field(rng, Nx, Ns)
    w = loopgen.random_band_field(rng, Nx, Ns)
    v2 = 0.37
    T = 31.0
    lhs = K.inner(K.directional_derivative(u, T, L, v1, v2), w, L)
    a1, a2 = K.adjoint_operator(u, T, L, w)
    rhs = K.inner(v1, a1, L) + v2 * a2
    mag = np.sqrt(l2(K.directional_derivative(u, T, L, v1, v2), L) * l2(w, L))
    assert abs(lhs - rhs) <= 1e-13 * mag


def test_adjoint_of_residual_is_the_flow():
    """G = -L^dagger(l; [r; 0]) (eq. G_as_adjoint)."""
    rng = np.random.default_rng(RNG_SEED)
    Nx, Ns, L, T = 32, 32, 22.0, 20.0
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=4, kmax=3, scale=0.5)
    r = K.residual(u, T, L)
    a1, a2 = K.adjoint_operator(u, T, L, r)
    G, dT, _ = K.adjoint_grad(u, T, L)
    assert rel(G, -a1) < 1e-13
    assert abs(dT - a2) < 1e-13 * abs(a2)


def test_directional_derivative_is_the_limit():
    """L(l; v) equals the limit defining it (eq. directional_derivative), by central differences."""
    rng = np.random.default_rng(RNG_SEED + 7)
    Nx, Ns, L, T = 32, 64, 22.0, 25.0
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=5, kmax=5, scale=0.5)
    v1 = loopgen.random_band_field(rng, Nx, Ns, jmax=5, kmax=5)
    v2 = 0.8
    h = 1e-5
    fd = (K.residual(u + h * v1, T + h * v2, L) - K.residual(u - h * v1, T - h * v2, L)) / (2 * h)
    an = K.directional_derivative(u, T, L, v1, v2)
    assert rel(fd, an) < 1e-7


# ------------------------------------------------------------------------------ pi4 finite differences
@pytest.mark.parametrize("Nx,Ns,L,T", [(32, 32, 22.0, 20.0), (32, 64, 39.0, 45.0)])
def test_gradient_matches_central_differences(Nx, Ns, L, T):
    rng = np.random.default_rng(RNG_SEED + 3)
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=4, kmax=3, scale=0.5, zero_mean=True)
    G, dT, J = K.adjoint_grad(u, T, L)
    h = 1e-6
    for trial in range(6):
        v1 = loopgen.random_band_field(rng, Nx, Ns)
        v2 = float(rng.standard_normal())
        nrm = np.sqrt(l2(v1, L) + v2 * v2)  # unit direction in the norm of eq. L2norm_definition
        v1, v2 = v1 / nrm, v2 / nrm
        Jp = K.cost(u + h * v1, T + h * v2, L)
        Jm = K.cost(u - h * v1, T - h * v2, L)
        fd = (Jp - Jm) / (2 * h)
        D = -(K.inner(G, v1, L) + (-dT) * v2)  # dJ = <grad J, v> = -<G, v>, with G_2 = -dJ/dT
        assert abs(fd - D) <= 1e-8 * max(abs(J), abs(D))


def test_period_derivative_matches_central_difference():
    rng = np.random.default_rng(RNG_SEED + 4)
    Nx, Ns, L, T = 32, 64, 22.0, 33.0
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=4, kmax=6, scale=0.5)
    h = 1e-5
    fd = (K.cost(u, T + h, L) - K.cost(u, T - h, L)) / (2 * h)
    assert abs(fd - K.dJdT(u, T, L)) < 1e-7 * max(abs(fd), 1e-3 * K.cost(u, T, L))


# ------------------------------------------------------------------------------ pi5 equivariance
def shift(uhat, L, a=0.0, sigma=0.0):
    Nx, Ns = 2 * (uhat.shape[1] - 1), uhat.shape[0]
    q, omega = K.wavenumbers(L, Nx, Ns)
    return uhat * np.exp(-1j * q * a) * np.exp(-1j * omega * sigma)


@pytest.mark.parametrize("a,sigma", [(1.2345, 0.0), (0.0, 0.3141), (2.7, 0.77)])
def test_shift_equivariance(a, sigma):
    rng = np.random.default_rng(RNG_SEED + 5)
    Nx, Ns, L, T = 32, 64, 22.0, 30.0
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=5, kmax=6, scale=0.5)
    G, dT, J = K.adjoint_grad(u, T, L)
    Gs, dTs, Js = K.adjoint_grad(shift(u, L, a, sigma), T, L)
    assert abs(Js - J) < 1e-13 * J
    assert abs(dTs - dT) < 1e-12 * max(abs(dT), 1e-3 * J)
    assert rel(Gs, shift(G, L, a, sigma)) < 1e-12


# ------------------------------------------------------------------------------ pi6 Xi symmetry
def xi(uhat):
    """Xi: (x, s) -> (-x, s), u -> -u, i.e. u_hat_{j,k} -> -conj(u_hat_{j,-k}) (eq. KS_loop_sym)."""
    Ns = uhat.shape[0]
    idx = (-np.arange(Ns)) % Ns
    return -np.conj(uhat[idx, :])


def test_xi_equivariance():
    rng = np.random.default_rng(RNG_SEED + 6)
    Nx, Ns, L, T = 32, 32, 39.0, 40.0
    u = K.canonical(loopgen.random_band_field(rng, Nx, Ns, jmax=6, kmax=6, scale=0.5))
    G, dT, J = K.adjoint_grad(u, T, L)
    Gx, dTx, Jx = K.adjoint_grad(xi(u), T, L)
    assert abs(Jx - J) < 1e-13 * J
    assert abs(dTx - dT) < 1e-12 * max(abs(dT), 1e-3 * J)
    assert rel(Gx, xi(G)) < 1e-13


def test_xi_invariant_loop_stays_invariant():
    rng = np.random.default_rng(RNG_SEED + 8)
    Nx, Ns, L, T = 32, 32, 39.0, 40.0
    u = loopgen.random_xi_symmetric_field(rng, Nx, Ns, jmax=6, kmax=5, scale=0.4)
    assert rel(xi(u), u) < 1e-15
    u1, T1, _ = K.step(u, T, L, 1e-4, K.IMEX, nsteps=20)
    assert rel(xi(u1), u1) < 1e-13
    assert np.max(np.abs(u1[:, 0])) < 1e-13 * np.max(np.abs(u1))  # the mean and column 0 stay zero


# ------------------------------------------------------------------------------ pi7 descent
def test_explicit_descent_monotone_and_rate():
    c = loopgen.config_loops(1)[0]
    u, T, Jh = K.step(c.uhat, c.T, c.L, 1e-4, K.EXPLICIT, nsteps=200)
    assert np.all(np.diff(Jh) <= 0.0)
    # first-order rate: (J(tau + dtau) - J) / dtau -> -||G||^2 (eq. J_variation with J halved)
    G, dT, J0 = K.adjoint_grad(c.uhat, c.T, c.L)
    rate = -(l2(G, c.L) + dT * dT)
    errs = []
    for dtau in (1e-6, 5e-7):
        u1, T1, _ = K.step(c.uhat, c.T, c.L, dtau, K.EXPLICIT, 1)
        errs.append(abs((K.cost(u1, T1, c.L) - J0) / dtau - rate))
    assert errs[0] < 1e-2 * abs(rate)
    assert 1.6 < errs[0] / errs[1] < 2.4  # error halves with dtau: first order


def test_imex_descent_monotone_and_rate():
    c = loopgen.config_loops(2)[0]
    u, T, Jh = K.step(c.uhat, c.T, c.L, 5e-5, K.IMEX, nsteps=60)
    assert np.all(np.diff(Jh) <= 0.0)
    G, dT, J0 = K.adjoint_grad(c.uhat, c.T, c.L)
    Nx, Ns = c.Nx, c.Ns
    dtau = 1e-9
    sig = 1.0 / (1.0 - dtau * K.lam(c.T, c.L, Nx, Ns))
    rate = -(K.inner(G, sig * G, c.L) + dT * dT)
    u1, T1, _ = K.step(c.uhat, c.T, c.L, dtau, K.IMEX, 1)
    assert abs((K.cost(u1, T1, c.L) - J0) / dtau - rate) < 1e-3 * abs(rate)


# ------------------------------------------------------------------------------ pi8 linear limit
def test_linear_limit():
    Nx, Ns, L, T = 32, 32, 22.0, 20.0
    rng = np.random.default_rng(RNG_SEED + 9)
    base = loopgen.random_band_field(rng, Nx, Ns, jmax=3, kmax=3, zero_mean=True)
    lm = K.lam(T, L, Nx, Ns)
    prev = None
    for A in (1e-3, 1e-4):
        u = A * base
        G, _, _ = K.adjoint_grad(u, T, L)
        err = np.max(np.abs(G - lm * u)) / np.max(np.abs(lm * u))
        if prev is not None:
            assert err < 0.2 * prev  # nonlinear remainder is O(A) relative
        prev = err
    assert prev < 1e-2
    # one step multiplies each mode by 1 + dtau*lam (explicit) or 1/(1 - dtau*lam) (IMEX)
    u = 1e-9 * base
    dtau = 1e-3
    ue, _, _ = K.step(u, T, L, dtau, K.EXPLICIT, 1)
    ui, _, _ = K.step(u, T, L, dtau, K.IMEX, 1)
    m = np.abs(u) > 0
    assert np.max(np.abs(ue[m] / u[m] - (1 + dtau * lm)[m])) < 1e-6
    assert np.max(np.abs(ui[m] / u[m] - (1 / (1 - dtau * lm))[m])) < 1e-6


# ------------------------------------------------------------------------------ pi9 fixed points
def test_constant_field_is_a_fixed_point():
    Nx, Ns, L = 32, 32, 22.0
    u = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    u[0, 0] = 1.7
    for T in (5.0, 50.0):
        G, dT, J = K.adjoint_grad(u, T, L)
        assert np.max(np.abs(K.residual(u, T, L))) == 0.0
        assert np.max(np.abs(G)) == 0.0 and dT == 0.0 and J == 0.0


def test_time_independent_field_has_zero_period_derivative():
    rng = np.random.default_rng(RNG_SEED + 10)
    Nx, Ns, L = 32, 32, 22.0
    u = loopgen.random_band_field(rng, Nx, Ns, jmax=5, kmax=0)
    _, dT, J = K.adjoint_grad(u, 20.0, L)
    assert J > 0 and dT == 0.0


# ------------------------------------------------------------------------------ boundary reading
def test_column0_reading_matches_real_inverse_transform():
    rng = np.random.default_rng(RNG_SEED + 11)
    Nx, Ns = 16, 16
    u = rng.standard_normal((Ns, Nx // 2 + 1)) + 1j * rng.standard_normal((Ns, Nx // 2 + 1))
    u = K.project(u)
    via_grid = K.project(K.from_grid(K.to_grid(u)))
    assert rel(K.canonical(u), via_grid) < 1e-14


def test_step_output_is_in_band_and_real():
    c = loopgen.config_loops(1)[0]
    u, T, _ = K.step(c.uhat, c.T, c.L, 1e-4, K.EXPLICIT, 3)
    assert np.all(u[~K.band_mask(c.Nx, c.Ns)] == 0)
    assert rel(K.hermitian_column0(u), u) < 1e-14


# ------------------------------------------------------------------------------ autograd convention
def torch_cost(u, T, L, Nx, Ns):
    """J = 1/2 int int r^2 written with torch.fft (CPU, FP64), differentiable in u and T."""
    import torch
    Kx, Ks = K.band_limits(Nx, Ns)
    j = torch.arange(Nx // 2 + 1, dtype=torch.float64)
    k = torch.fft.fftfreq(Ns, d=1.0 / Ns, dtype=torch.float64)
    mask = ((k.abs()[:, None] <= Ks) & (j[None, :] <= Kx)).to(torch.complex128)
    q = (2 * np.pi * j / L)[None, :].to(torch.complex128)
    om = (2 * np.pi * k)[:, None].to(torch.complex128)
    u = u * mask
    g = lambda v: torch.fft.irfft2(v, s=(Ns, Nx), norm="forward")
    r = -g(1j * om * u) / T - g(u) * g(1j * q * u) - g(-(q ** 2) * u) - g(q ** 4 * u)
    r = g(torch.fft.rfft2(r, norm="forward") * mask)
    return 0.5 * L * torch.mean(r * r)


def test_autograd_grad_matches_torch_autograd():
    """grad = -w_j L G_1 and dJ/dT in torch's complex convention (reading R11), against
    torch's own autograd through torch.fft, including a non-Hermitian column 0 and
    out-of-band entries in the input."""
    import torch
    rng = np.random.default_rng(RNG_SEED + 12)
    Nx, Ns, L, T = 16, 32, 13.0, 17.0
    u0 = loopgen.random_band_field(rng, Nx, Ns, scale=0.5)
    u0 = u0 + 0.2 * (rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape))
    ut = torch.tensor(u0, requires_grad=True)
    Tt = torch.tensor(T, dtype=torch.float64, requires_grad=True)
    J = torch_cost(ut, Tt, L, Nx, Ns)
    J.backward()
    g_u, g_T = K.autograd_grad(u0, T, L)
    assert abs(J.item() - K.cost(u0, T, L)) < 1e-13 * J.item()
    assert np.max(np.abs(ut.grad.numpy() - g_u)) < 1e-12 * np.max(np.abs(g_u))
    assert abs(Tt.grad.item() - g_T) < 1e-12 * max(abs(g_T), 1e-3 * J.item())


def test_xi_project_is_the_orthogonal_projection_onto_invariant_loops():
    """xi_project (the invariant part (u + Xi u) / 2) is idempotent, lands in the invariant
    loops, fixes them, is orthogonal in the inner product of eq. inner_product_definition,
    and identifies u with Xi u."""
    rng = np.random.default_rng(17)
    L = 22.0
    for (Nx, Ns) in [(16, 16), (32, 64), (64, 32)]:
        u = loopgen.random_band_field(rng, Nx, Ns)
        P = K.xi_project(u)
        assert rel(K.xi_project(P), P) < 1e-15
        assert rel(xi(P), P) < 1e-15
        v = loopgen.random_xi_symmetric_field(rng, Nx, Ns)
        assert rel(K.xi_project(v), v) < 1e-15
        assert abs(K.inner(u - P, P, L)) < 1e-13 * K.inner(u, u, L)
        assert abs(K.inner(u - P, v, L)) < 1e-13 * np.sqrt(K.inner(u, u, L) * K.inner(v, v, L))
        assert rel(K.xi_project(xi(u)), P) < 1e-15
        assert np.all(P[:, 0] == 0)
