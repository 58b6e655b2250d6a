"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch each one.

Each mutation monkeypatches one piece of the transform-based oracle, for example a dropped
term, a flipped sign or a wrong operand. The test then checks that at least one of the pin
tests in ``test_oracle.py`` fails on the mutated oracle.
"""
import numpy as np
import pytest

from oracle import ks_loop as K

import test_oracle as P

PINS = [
    lambda: P.test_brute_force_matches_transform_oracle(16, 12),
    lambda: P.test_single_mode_closed_form(2, 3),
    lambda: P.test_single_mode_closed_form(0, 3),
    lambda: P.test_gradient_matches_central_differences(32, 32, 22.0, 20.0),
    lambda: P.test_imex_descent_monotone_and_rate(),
    lambda: P.test_linear_limit(),
    lambda: P.test_adjoint_identity(16, 16, 7.0),
    lambda: P.test_adjoint_of_residual_is_the_flow(),
    lambda: P.test_directional_derivative_is_the_limit(),
]


def _any_pin_fails():
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            return True
    return False


def _mut_residual_sign_us(uhat, T, L):
    u = K.canonical(uhat)
    r = +(1.0 / T) * K.d_s(u, L) - K.product(u, K.d_x(u, L)) - K.d_xx(u, L) - K.d_xxxx(u, L)
    return K.project(r)


def _mut_residual_drop_uxx(uhat, T, L):
    u = K.canonical(uhat)
    r = -(1.0 / T) * K.d_s(u, L) - K.product(u, K.d_x(u, L)) - K.d_xxxx(u, L)
    return K.project(r)


def _mut_grad_wrong_operand(uhat, T, L):
    u = K.canonical(uhat)
    r = K.residual(u, T, L)
    G = -(1.0 / T) * K.d_s(r, L) - K.product(r, K.d_x(u, L)) + K.d_xx(r, L) + K.d_xxxx(r, L)
    rg = K.to_grid(r)
    J = 0.5 * K.space_time_integral(rg * rg, L)
    dT = K.space_time_integral(K.to_grid(K.d_s(u, L)) * rg / (T * T), L)
    return K.project(G), dT, J


def _mut_grad_sign_rs(uhat, T, L):
    u = K.canonical(uhat)
    r = K.residual(u, T, L)
    G = +(1.0 / T) * K.d_s(r, L) - K.product(u, K.d_x(r, L)) + K.d_xx(r, L) + K.d_xxxx(r, L)
    rg = K.to_grid(r)
    J = 0.5 * K.space_time_integral(rg * rg, L)
    dT = K.space_time_integral(K.to_grid(K.d_s(u, L)) * rg / (T * T), L)
    return K.project(G), dT, J


def _mut_grad_dT_power(uhat, T, L):
    G, dT, J = _orig_adjoint_grad(uhat, T, L)
    return G, dT * T, J  # 1/T instead of 1/T^2


def _mut_grad_J_no_half(uhat, T, L):
    G, dT, J = _orig_adjoint_grad(uhat, T, L)
    return G, dT, 2 * J


def _mut_wavenumbers_no_L(L, Nx, Ns):
    q, w = _orig_wavenumbers(L, Nx, Ns)
    return q * L / (2 * np.pi) * 2 * np.pi, w


def _mut_lam_sign(T, L, Nx, Ns):
    return -_orig_lam(T, L, Nx, Ns)


def _mut_no_hermitian(vhat):
    return np.array(vhat, dtype=np.complex128, copy=True)


def _mut_band_off_by_one(Nx, Ns):
    return (Nx - 1) // 3 + 1, (Ns - 1) // 3


_orig_adjoint_grad = K.adjoint_grad
_orig_wavenumbers = K.wavenumbers
_orig_lam = K.lam

MUTATIONS = [
    ("residual", _mut_residual_sign_us),
    ("residual", _mut_residual_drop_uxx),
    ("adjoint_grad", _mut_grad_wrong_operand),
    ("adjoint_grad", _mut_grad_sign_rs),
    ("adjoint_grad", _mut_grad_dT_power),
    ("adjoint_grad", _mut_grad_J_no_half),
    ("wavenumbers", _mut_wavenumbers_no_L),
    ("lam", _mut_lam_sign),
    ("hermitian_column0", _mut_no_hermitian),
    ("band_limits", _mut_band_off_by_one),
]


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[f"{n}-{f.__name__}" for n, f in MUTATIONS])
def test_pins_catch_planted_mistake(monkeypatch, name, fn):
    monkeypatch.setattr(K, name, fn)
    assert _any_pin_fails(), f"no pin caught the mutation {fn.__name__}"


def test_pins_pass_unmutated():
    assert not _any_pin_fails()
