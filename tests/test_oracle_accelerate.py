"""Pins of the oracle's convergence driver with the extrapolations of App. C.

* The extrapolation formula recovers the fixed point of an exactly geometric sequence.
* A single Fourier mode whose products fall outside the two-thirds band evolves exactly
  linearly (IMEX: u <- u / (1 - dtau lambda) each step), so one extrapolation must land on
  the fixed point u = 0 to rounding.
* On a nonlinear loop the accelerated run needs fewer steps and ends on the same state as
  the plain run (up to the period, which the flow leaves free on an equilibrium).
"""
import numpy as np

import loopgen
from oracle import accelerate as A
from oracle import ks_loop as K


def test_extrapolation_of_a_geometric_sequence_is_exact():
    rng = np.random.default_rng(0)
    ustar = loopgen.random_band_field(rng, 16, 16)
    v = loopgen.random_band_field(rng, 16, 16)
    Tstar, vT = 31.0, 0.7
    for rho in (0.5, 0.3, 0.9):
        ua, Ta = ustar + 1e-3 * v, Tstar + 1e-3 * vT
        ub, Tb = ustar + rho * 1e-3 * v, Tstar + rho * 1e-3 * vT
        u, T = A.extrapolate(ua, Ta, ub, Tb, rho)
        assert np.abs(u - ustar).max() <= 1e-14 * np.abs(ustar).max()
        assert abs(T - Tstar) <= 1e-13 * Tstar


def test_single_mode_linear_dynamics_one_extrapolation_lands_on_zero():
    Nx, Ns, L = 8, 8, 22.0
    u0 = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    u0[0, 2] = 0.05  # u = 0.1 cos(2 q x): u u_x has |j| = 4, outside the band |j| <= 2
    T0 = 25.0
    # the plain run decays geometrically; J after one IMEX step is exactly g^2 J before it
    q = 2 * np.pi * 2 / L
    lam = -q ** 8 + 2 * q ** 6 - q ** 4
    g = 1.0 / (1.0 - 1.0 * lam)
    u1, T1, Jh = K.step(u0, T0, L, 1.0, K.IMEX, 3)
    assert np.allclose(Jh[1:] / Jh[:-1], g * g, rtol=1e-13, atol=0)
    assert T1 == T0  # time independent: dJ/dT = 0
    u, T, J, steps, ext = A.converge(u0, T0, L, 1.0, K.IMEX, 1e-24, 1, 1000, True, sqrtJ_first=1.0)
    assert ext == 1
    assert J < 1e-28 * K.cost(u0, T0, L)
    assert np.abs(u).max() < 1e-14 * 0.05
    assert steps < 30  # sqrt(J) halves in log(2) / log(1/g) steps


def test_accelerated_run_saves_steps_and_reaches_the_same_state():
    s = loopgen.random_loop(5, 14.0, 16, 16, 2, 2, 0.8, 0.3, 20.0)
    up, Tp, Jp, np_, ep = A.converge(s.uhat, s.T, s.L, 0.1, K.IMEX, 1e-10, 20, 60000, False)
    ua, Ta, Ja, na, ea = A.converge(s.uhat, s.T, s.L, 0.1, K.IMEX, 1e-10, 20, 60000, True)
    assert ep == 0 and ea >= 1
    assert Jp < 1e-10 and Ja < 1e-10
    assert na < 0.8 * np_
    norm = np.sqrt(K.inner(up, up, s.L))
    assert norm > 0.5  # a non-trivial end state
    # same state up to the free period and shifts: band-mode magnitudes agree. Both end states
    # have sqrt(J) < 1e-5, so each lies O(1e-5) from the equilibrium (a stopping criterion on
    # J, not on the state); the tolerance is 5e-5 of the norm.
    assert np.abs(np.abs(ua) - np.abs(up)).max() < 5e-5 * norm
