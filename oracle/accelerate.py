"""Convergence driver of the loop dynamics, with the acceleration of App. C.

TEST INFRASTRUCTURE. The parity reference for the device convergence driver; only the test
suite and the stored-fixture script use it. It shares no code with the HIP library.

App. C (acceleration by a linearised approximation): time stepping of eq. KS_G alternates
with linear extrapolations of the loop along its trajectory. Near the attracting fixed point
the loop approaches it along the leading eigendirection of the linearised loop dynamics. The
first extrapolation is made once sqrt(J) has come down to 1e-3. Between two extrapolations the
loop is advanced until sqrt(J) has halved.

The appendix gives no formula; the readings taken here:

* Extrapolation. Near the fixed point l*, l(tau) - l* ~ c exp(-mu tau) v and sqrt(J) is
  proportional to |l - l*|. Two states l_a, l_b on the trajectory with sqrt(J_b) = rho
  sqrt(J_a) then give l* = l_b + rho / (1 - rho) (l_b - l_a). It is applied to the whole loop,
  (u_hat, T), alike.
* Intervals. The first interval starts at the first examined state with sqrt(J) <= 1e-3;
  each later one starts at the extrapolated state. An interval ends at the first examined
  state whose sqrt(J) is at most half the value at its start, and the extrapolation is made
  from the interval's two end states.
* Which J. J here is half the paper's (J = 1/2 int int r^2), and both thresholds are applied
  to sqrt of this J. The halving test and rho are ratios, so the factor drops out of them.
  The start test sqrt(J) <= sqrtJ_first is the paper's sqrt(J_paper) <= 1e-3 when
  sqrtJ_first = 1e-3 / sqrt(2); the default 1e-3 starts a little later, at
  sqrt(J_paper) <= sqrt(2) 1e-3. The device driver (loop_converge) takes the same argument.
* Examination. J is examined on the state after every `stride` steps (and on the initial
  state), so that a device implementation that runs `stride` steps per launch takes the same
  decisions. The run stops at the first examined state with J < J_tol, or after max_steps.
"""
from __future__ import annotations

import math

import numpy as np

from . import ks_loop as K


def extrapolate(ua: np.ndarray, Ta: float, ub: np.ndarray, Tb: float, rho: float):
    """l_b + rho / (1 - rho) (l_b - l_a) for l = (u_hat, T), rho = sqrt(J_b / J_a) < 1."""
    f = rho / (1.0 - rho)
    return ub + f * (ub - ua), Tb + f * (Tb - Ta)


def converge(uhat: np.ndarray, T: float, L: float, dtau: float, scheme: int, J_tol: float, stride: int,
             max_steps: int, accelerate: bool, sqrtJ_first: float = 1e-3):
    """Advance the loop until J < J_tol (examined every `stride` steps), with or without the
    extrapolations of App. C. Returns (u_hat, T, J, steps, extrapolations)."""
    u = K.canonical(uhat)
    J = K.cost(u, T, L)
    steps = 0
    extraps = 0
    anchor = None  # (u, T, J) at the start of the current interval
    while J >= J_tol and steps < max_steps:
        u, T, _ = K.step(u, T, L, dtau, scheme, stride)
        steps += stride
        J = K.cost(u, T, L)
        if not accelerate or J < J_tol:
            continue
        if anchor is None:
            if math.sqrt(J) <= sqrtJ_first:
                anchor = (u, T, J)
        elif math.sqrt(J) <= 0.5 * math.sqrt(anchor[2]):
            rho = math.sqrt(J / anchor[2])
            u, T = extrapolate(anchor[0], anchor[1], u, T, rho)
            extraps += 1
            J = K.cost(u, T, L)
            anchor = (u, T, J)
    return u, T, J, steps, extraps
