"""Pins of the oracle's expanded form of the flow (oracle/ks_loop.py expanded_grad and
step_expanded; Sec. 4.2, eq. KS_G_1) and the planted mistakes they catch.

The expanded form and the residual-then-adjoint form (pinned in test_oracle.py) are the same
flow in the continuum. On the grid they agree to round-off whenever no product leaves the
band before it is used and none aliases into it: for modes |j| <= jm, |k| <= km with 2 jm <= Kx,
2 km <= Ks (r lies in the band) and 3 jm + Kx < Nx, 3 km + Ks < Ns (the cubic products do not
alias into the band). dJ/dT agrees for every band-limited loop, since u_s r has no aliased
mean."""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def low_mode_loop(rng, Nx, Ns, scale=0.5):
    Kx, Ks = K.band_limits(Nx, Ns)
    return loopgen.random_band_field(rng, Nx, Ns, jmax=Kx // 2, kmax=Ks // 2, scale=scale)


CASES = [(16, 16, 22.0, 20.0), (32, 64, 22.0, 35.0), (64, 32, 39.0, 59.0), (64, 128, 39.0, 80.0)]


@pytest.mark.parametrize("Nx,Ns,L,T", CASES)
def test_expanded_equals_adjoint_form_where_nothing_is_truncated(Nx, Ns, L, T):
    rng = np.random.default_rng(Nx + Ns)
    u = low_mode_loop(rng, Nx, Ns)
    Ga, dTa, Ja = K.adjoint_grad(u, T, L)
    Ge, dTe, Je = K.expanded_grad(u, T, L)
    assert rel(Ge, Ga) < 1e-13
    assert abs(dTe - dTa) <= 1e-13 * abs(dTa)
    assert abs(Je - Ja) <= 1e-13 * Ja


@pytest.mark.parametrize("Nx,Ns,L,T", CASES)
def test_period_derivative_agrees_on_full_band_loops(Nx, Ns, L, T):
    rng = np.random.default_rng(3 * Nx + Ns)
    u = loopgen.random_band_field(rng, Nx, Ns, scale=0.5)
    _, dTa, Ja = K.adjoint_grad(u, T, L)
    Ge, dTe, Je = K.expanded_grad(u, T, L)
    assert abs(dTe - dTa) <= 1e-12 * max(abs(dTa), 1e-3 * Ja)
    assert Je >= Ja * (1 - 1e-12)  # the grid residual adds the out-of-band part of u u_x


def test_linear_part_is_lambda_u():
    """For amplitude eps the expanded G is lambda u_hat + O(eps^2)."""
    rng = np.random.default_rng(5)
    Nx, Ns, L, T = 32, 32, 22.0, 30.0
    u = loopgen.random_band_field(rng, Nx, Ns, scale=1.0)
    lm = K.lam(T, L, Nx, Ns)
    d = []
    for eps in (1e-3, 5e-4):
        G, _, _ = K.expanded_grad(eps * u, T, L)
        d.append(np.max(np.abs(G - lm * K.canonical(eps * u))))
    assert 3.5 < d[0] / d[1] < 4.5


@pytest.mark.parametrize("scheme", [K.EXPLICIT, K.IMEX])
def test_expanded_step_equals_step_where_nothing_is_truncated(scheme):
    rng = np.random.default_rng(7)
    Nx, Ns, L, T = 64, 64, 39.0, 50.0
    u = low_mode_loop(rng, Nx, Ns, scale=0.2)
    dtau = 1e-4 if scheme == K.EXPLICIT else 0.05
    ua, Ta, Ja = K.step(u, T, L, dtau, scheme, 1)
    ue, Te, Je = K.step_expanded(u, T, L, dtau, scheme, 1)
    assert rel(ue, ua) < 1e-13 and abs(Te - Ta) < 1e-13 * Ta and abs(Je[0] - Ja[0]) < 1e-13 * Ja[0]


def test_truncation_difference_shrinks_with_the_spectrum():
    """On full-band loops the two forms differ; the difference falls with the spectral decay."""
    Nx, Ns, L, T = 64, 64, 22.0, 30.0
    diffs = []
    for beta in (0.2, 0.5, 1.0, 1.5):
        u = loopgen.seeded_spectrum(np.random.default_rng(11), Nx, Ns, 21, 21, 0.5, beta)
        Ga, _, _ = K.adjoint_grad(u, T, L)
        Ge, _, _ = K.expanded_grad(u, T, L)
        diffs.append(rel(Ge, Ga))
    assert diffs[0] > diffs[1] > diffs[2] > diffs[3] and diffs[0] > 1e-5 and diffs[3] < 1e-11


# ---------------------------------------------------------------- planted mistakes
def _mutant(c5=-5.0, c10=-10.0, c3=-3.0, c_uuxx=1.0, c_uux2=1.0, c_uxs=2.0, c_uxus=1.0, lin_sign=1.0):
    def f(uhat, T, L):
        u = K.canonical(uhat)
        Nx, Ns = K._shape(u)
        g = K.to_grid
        U, Ux, Uxx = g(u), g(K.d_x(u, L)), g(K.d_xx(u, L))
        Uxxx, Uxxxx = g(K.d_x(K.d_xx(u, L), L)), g(K.d_xxxx(u, L))
        Us, Uxs = g(K.d_s(u, L)), g(K.d_x(K.d_s(u, L), L))
        nl = (c5 * Uxxxx * Ux + c10 * Uxxx * Uxx + c3 * Uxx * Ux + c_uuxx * U * U * Uxx + c_uux2 * U * Ux * Ux
              + (c_uxs / T) * U * Uxs + (c_uxus / T) * Ux * Us)
        G = lin_sign * K.lam(T, L, Nx, Ns) * u + K.project(K.from_grid(nl))
        r = -(1.0 / T) * Us - U * Ux - Uxx - Uxxxx
        return K.project(G), K.space_time_integral(Us * r / (T * T), L), 0.5 * K.space_time_integral(r * r, L)
    return f


@pytest.mark.parametrize("kw", [{"c5": 5.0}, {"c10": -5.0}, {"c3": 3.0}, {"c_uuxx": -1.0}, {"c_uux2": 0.0},
                                {"c_uxs": 1.0}, {"c_uxus": -1.0}, {"lin_sign": -1.0}])
def test_pins_catch_planted_mistakes(monkeypatch, kw):
    u = loopgen.random_band_field(np.random.default_rng(1), 16, 16)
    same, ref = _mutant()(u, 20.0, 22.0), K.expanded_grad(u, 20.0, 22.0)
    assert np.array_equal(same[0], ref[0]) and same[1:] == ref[1:]  # the unmutated copy is the oracle
    monkeypatch.setattr(K, "expanded_grad", _mutant(**kw))
    with pytest.raises(AssertionError):
        for case in CASES:
            test_expanded_equals_adjoint_form_where_nothing_is_truncated(*case)
