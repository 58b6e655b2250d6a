"""Write the stored trajectory fixtures under tests/golden/ from the CPU oracle alone.

Run from the repository root:  python tests/golden/make_golden.py [plain64x128]
(the argument writes the 64 x 128 log alone). It imports only the oracle and the seeded input
generator.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import loopgen  # noqa: E402
from oracle import accelerate as A  # noqa: E402
from oracle import ks_loop as K  # noqa: E402


def band_list(u, Nx, Ns):
    Kx, Ks = K.band_limits(Nx, Ns)
    out = []
    for j in range(Kx + 1):
        for k in range(-Ks, Ks + 1):
            v = u[k % Ns, j]
            out.append([j, k, float(v.real), float(v.imag)])
    return out


def trajectory(c, steps, scheme, dtau, marks):
    spec = loopgen.config_loops(c)[0]
    u, T, Jh = K.step(spec.uhat, spec.T, spec.L, dtau, scheme, steps)
    return {
        "workload": loopgen.CONFIGS[c]["name"], "seed": spec.seed, "L": spec.L, "Nx": spec.Nx,
        "Ns": spec.Ns, "T0": spec.T, "dtau": dtau, "scheme": "imex" if scheme == K.IMEX else "explicit",
        "steps": steps, "J_hist_marks": {str(m): float(Jh[m]) for m in marks},
        "T_final": float(T), "uhat_final_band": band_list(u, spec.Nx, spec.Ns),
    }


def logged(c, steps, scheme, dtau, every):
    """Workload c's seed run for `steps` steps, with J and T logged at the start of every
    `every`-th step (J(tau) and T(tau) at tau = n dtau, n = 0, every, 2 every, ...) and the
    final state."""
    spec = loopgen.config_loops(c)[0]
    u, T = spec.uhat, spec.T
    J_log, T_log = [], []
    for _ in range(steps // every):
        T_log.append(float(T))
        u, T, Jh = K.step(u, T, spec.L, dtau, scheme, every)
        J_log.append(float(Jh[0]))
    return {
        "workload": loopgen.CONFIGS[c]["name"], "seed": spec.seed, "L": spec.L, "Nx": spec.Nx,
        "Ns": spec.Ns, "T0": spec.T, "dtau": dtau, "scheme": "imex" if scheme == K.IMEX else "explicit",
        "steps": steps, "log_every": every, "J_log": J_log, "T_log": T_log,
        "J_final": float(K.cost(u, T, spec.L)), "T_final": float(T), "uhat_final_band": band_list(u, spec.Nx, spec.Ns),
    }


def converged(c, dtau, scheme, jtol, chunk):
    """Run the oracle from workload c's seed, chunk steps at a time, until J < jtol at a chunk
    end. Records the step count, the end state's period, cost, band-mode magnitudes (which an
    x- or s-shift leaves alone) and how far the end state is from time independence."""
    spec = loopgen.config_loops(c)[0]
    u, T = spec.uhat, spec.T
    n = 0
    while True:
        u, T, _ = K.step(u, T, spec.L, dtau, scheme, chunk)
        n += chunk
        J = K.cost(u, T, spec.L)
        if J < jtol:
            break
    uc = K.canonical(u)
    norm_u = float(np.sqrt(K.inner(uc, uc, spec.L)))
    us = K.d_s(uc, spec.L)
    norm_us = float(np.sqrt(K.inner(us, us, spec.L)))
    kind = "equilibrium" if norm_us < 1e-3 * norm_u else ("trivial" if norm_u < 1e-6 else "periodic orbit")
    return {
        "workload": loopgen.CONFIGS[c]["name"], "seed": spec.seed, "L": spec.L, "Nx": spec.Nx, "Ns": spec.Ns,
        "T0": spec.T, "dtau": dtau, "scheme": "imex" if scheme == K.IMEX else "explicit", "J_tol": jtol,
        "steps": n, "T_final": float(T), "J_final": float(J), "norm_u": norm_u, "norm_u_s": norm_us,
        "end_state": kind, "abs_uhat_final_band": [[j, k, abs(complex(re, im))]
                                                   for j, k, re, im in band_list(u, spec.Nx, spec.Ns)],
    }


def driven(c, dtau, scheme, jtol, stride, accelerate):
    """The convergence driver of App. C (oracle/accelerate.py) from workload c's seed."""
    spec = loopgen.config_loops(c)[0]
    u, T, J, steps, ext = A.converge(spec.uhat, spec.T, spec.L, dtau, scheme, jtol, stride, 10 ** 6, accelerate)
    return {"accelerate": accelerate, "steps": steps, "extrapolations": ext, "T_final": float(T), "J_final": float(J),
            "abs_uhat_final_band": [[j, k, abs(complex(re, im))] for j, k, re, im in band_list(u, spec.Nx, spec.Ns)]}


def main(only=None):
    if only == "plain64x128":
        data = logged(2, 20000, K.IMEX, 5e-5, 10)
        with open(os.path.join(HERE, "oracle_traj_plain64x128.json"), "w") as f:
            json.dump(data, f)
        return
    data = trajectory(1, 2000, K.EXPLICIT, 1e-4, [0, 1, 10, 100, 1000, 1999])
    with open(os.path.join(HERE, "oracle_traj_plain32x32.json"), "w") as f:
        json.dump(data, f, indent=1)
    data = trajectory(2, 200, K.IMEX, 5e-5, [0, 1, 10, 100, 199])
    data.pop("uhat_final_band")
    with open(os.path.join(HERE, "oracle_traj_plain64x128_200.json"), "w") as f:
        json.dump(data, f, indent=1)
    data = logged(2, 20000, K.IMEX, 5e-5, 10)
    with open(os.path.join(HERE, "oracle_traj_plain64x128.json"), "w") as f:
        json.dump(data, f)
    data = converged(1, 0.05, K.IMEX, 1e-10, 2000)
    with open(os.path.join(HERE, "oracle_converged_plain32x32.json"), "w") as f:
        json.dump(data, f, indent=1)
    spec = loopgen.config_loops(1)[0]
    data = {"workload": loopgen.CONFIGS[1]["name"], "seed": spec.seed, "L": spec.L, "Nx": spec.Nx, "Ns": spec.Ns,
            "T0": spec.T, "dtau": 0.05, "scheme": "imex", "J_tol": 1e-10, "stride": 100, "sqrtJ_first": 1e-3,
            "runs": [driven(1, 0.05, K.IMEX, 1e-10, 100, False), driven(1, 0.05, K.IMEX, 1e-10, 100, True)]}
    with open(os.path.join(HERE, "oracle_accelerated_plain32x32.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else None)
