"""Write a converged orbit at L = 39 (tests/golden/oracle_orbit_L39*.json) with the oracle alone (Sec. 4.3-4.4).

The initial-loop pipeline of Sec. 4.3 and the loop dynamics, both from oracle/: centre-symmetric
chaotic KS runs at L = 39 (64 modes, ETDRK4, dt = 0.05, seeded small odd fields,
loopgen.random_ks_state with numpy.random.default_rng(2020), 200 time units of transient,
1000 recorded and sampled every 0.1), the first two norm-recurrence pairs of each run (1%,
20 <= T <= 160), their 64 x 64 loops (temporal modes |k| <= 10), and, for the loops whose
initial period lies in [23, 28], the accelerated convergence driver (IMEX, dtau = 0.15 as in
Sec. 4.4, J examined every 1000 steps, J < 1e-20). The first loop that converges is stored:
its initial spectrum, and its converged period, cost, step and extrapolation counts and state
(a loop at the paper's T = 25.37 first, if one converged there).

    python tests/golden/make_orbit.py            (about 15 minutes on 8 cores)
    python tests/golden/make_orbit.py LO HI TARGET MAX_STEPS OUT.json [J_TOL]
        (another window of initial periods, preferring an orbit at period TARGET)

The stored fixtures:

    oracle_orbit_L39.json       python tests/golden/make_orbit.py
    oracle_orbit_L39_T76.json   python tests/golden/make_orbit.py 76.0 76.5 76.61 4000000 oracle_orbit_L39_T76.json 5e-20
                                (about 65 minutes: three loops of 2.7-3.8 million steps each)
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import loopgen  # noqa: E402
from oracle import accelerate as A  # noqa: E402
from oracle import ks_dns as D  # noqa: E402
from oracle import ks_loop as K  # noqa: E402

L, NX, DT, EVERY, NS, KC = 39.0, 64, 0.05, 2, 64, 10
DTAU, J_TOL, STRIDE, MAX_STEPS = 0.15, 1e-20, 1000, 800_000
T_WINDOW = (23.0, 28.0)
TARGET = 25.37
OUT = "oracle_orbit_L39.json"
if len(sys.argv) in (6, 7):
    T_WINDOW = (float(sys.argv[1]), float(sys.argv[2]))
    TARGET, MAX_STEPS, OUT = float(sys.argv[3]), int(sys.argv[4]), sys.argv[5]
    if len(sys.argv) == 7:
        J_TOL = float(sys.argv[6])


def run_candidates(r_u0):
    r, u0 = r_u0
    u, _, _ = D.integrate(u0, L, DT, 4000, 4000, symmetric=True)
    _, n, s = D.integrate(u, L, DT, 20000, EVERY, symmetric=True)
    out = []
    for (a, b) in D.recurrences(n, DT * EVERY, 0.01, 20.0, 160.0)[:2]:
        loop, T = D.segment_to_loop(s, a, b, DT * EVERY, NS, KC)
        out.append((r, a, b, loop, T))
    return out


def converge(c):
    r, a, b, loop, T0 = c
    u, T, J, steps, ex = A.converge(loop, T0, L, DTAU, K.IMEX, J_TOL, STRIDE, MAX_STEPS, True)
    return r, a, b, T0, u, T, J, steps, ex


def main():
    rng = np.random.default_rng(2020)
    u0s = [(r, loopgen.random_ks_state(rng, NX, scale=0.1, odd=True)) for r in range(64)]
    with mp.Pool(8) as pool:
        cands = [c for cs in pool.map(run_candidates, u0s) for c in cs]
        pick = [c for c in cands if T_WINDOW[0] <= c[4] <= T_WINDOW[1]]
        print(f"{len(cands)} loops, {len(pick)} with T0 in {T_WINDOW}", flush=True)
        results = pool.map(converge, pick)
    for (r, a, b, T0, u, T, J, steps, ex), c in zip(results, pick):
        print(f"run {r} samples {a}..{b}: T0 {T0:.2f} -> T {T:.6f}, J {J:.3e}, {steps} steps, {ex} extrapolations",
              flush=True)
    done = [(res, c) for res, c in zip(results, pick) if res[6] < J_TOL]
    if not done:
        raise SystemExit("no loop converged")
    # prefer the orbit the paper reports at T = TARGET (Fig. 5) if one of them reached it
    done.sort(key=lambda rc: abs(rc[0][5] - TARGET) > 0.02)
    (r, a, b, T0, u, T, J, steps, ex), c = done[0]
    loop = c[3]
    Kx, Ks = K.band_limits(NX, NS)
    init = [[j, k, float(loop[k % NS, j].real), float(loop[k % NS, j].imag)]
            for k in range(-KC, KC + 1) for j in range(0, Kx + 1) if loop[k % NS, j] != 0]
    final = [[j, k, float(u[k % NS, j].real), float(u[k % NS, j].imag)]
             for k in range(-Ks, Ks + 1) for j in range(0, Kx + 1)]
    out = {
        "recipe": __doc__.strip().splitlines()[0],
        "command": " ".join(["python", "tests/golden/make_orbit.py"] + sys.argv[1:]), "L": L, "Nx": NX, "Ns": NS, "dtau": DTAU, "scheme": "imex",
        "J_tol": J_TOL, "stride": STRIDE, "max_steps": MAX_STEPS, "sqrtJ_first": 1e-3,
        "run": r, "samples": [a, b], "T0": T0, "uhat0_modes": init,
        "T_final": T, "J_final": J, "steps": steps, "extrapolations": ex, "uhat_final_band": final,
    }
    json.dump(out, open(os.path.join(HERE, OUT), "w"))
    print(f"stored run {r}: T = {T:.6f}", flush=True)


if __name__ == "__main__":
    main()
