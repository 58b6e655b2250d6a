"""Checks against stored fixtures under tests/golden/.

* paper_facts.json: statements the paper makes that can be exercised on synthetic loops.
  Currently this is the stability of the semi-implicit step at the paper's dtau (Sec. 4.2).
* oracle_traj_*.json: trajectories written by tests/golden/make_golden.py from the oracle
  alone. This is a regression pin that keeps the oracle fixed across edits.
"""
import json
import os

import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(HERE, name)) as f:
        return json.load(f)


def test_paper_dtau_is_stable_for_imex_at_paper_resolution():
    facts = load("paper_facts.json")
    Nx, Ns = facts["modes"]["value"]
    L = facts["L_chaotic"]["value"]
    dtau = facts["dtau_stable_imex"]["value"]
    rng = np.random.default_rng(777)
    # The paper's loops are smooth guesses near the orbit set; synthetic loops of O(1) amplitude
    # exceed the explicit nonlinear part's own step limit at this dtau. A small-amplitude loop
    # checks the claim where it is a statement about the scheme: the implicit linear part
    # damps every mode (0 < 1/(1 - dtau lambda) <= 1), where explicit Euler would not.
    u = loopgen.seeded_spectrum(rng, Nx, Ns, 6, 6, 0.05, 0.2)
    u1, T1, Jh = K.step(u, 40.0, L, dtau, K.IMEX, nsteps=150)
    assert np.all(np.isfinite(Jh)) and np.isfinite(T1)
    assert Jh[-1] < 0.1 * Jh[0] and np.all(np.diff(Jh) <= 0)
    lm = K.lam(40.0, L, Nx, Ns)
    assert dtau * np.max(np.abs(lm[K.band_mask(Nx, Ns)])) > 2.0  # explicit would be unstable
    ue, Te, Jhe = K.step(u, 40.0, L, dtau, K.EXPLICIT, nsteps=40)
    assert not (np.all(np.isfinite(Jhe)) and Jhe[-1] < Jhe[0])


def test_oracle_trajectory_regression_plain32x32():
    g = load("oracle_traj_plain32x32.json")
    spec = loopgen.config_loops(1)[0]
    assert spec.seed == g["seed"] and spec.T == g["T0"]
    u, T, Jh = K.step(spec.uhat, spec.T, spec.L, g["dtau"], K.EXPLICIT, g["steps"])
    for m, v in g["J_hist_marks"].items():
        assert abs(Jh[int(m)] - v) <= 1e-12 * abs(v)
    assert abs(T - g["T_final"]) <= 1e-12 * abs(T)
    for j, k, re, im in g["uhat_final_band"]:
        assert abs(u[k % spec.Ns, j] - complex(re, im)) <= 1e-12 * (1 + abs(complex(re, im)))


def test_oracle_log_plain64x128_prefix_and_descent():
    """The 64 x 128 workload's 20 000-step IMEX log (J and T every 10 steps): the oracle
    reproduces its first 2000 steps, J never increases along it (the flow descends J, eq.
    J_variation) and T moves by the explicit Euler steps of dJ/dT, which this flow keeps small."""
    g = load("oracle_traj_plain64x128.json")
    spec = loopgen.config_loops(2)[0]
    assert spec.seed == g["seed"] and spec.T == g["T0"] and g["log_every"] == 10 and len(g["J_log"]) == 2000
    u, T = spec.uhat, spec.T
    for i in range(200):
        assert abs(T - g["T_log"][i]) <= 1e-12 * abs(T)
        u, T, Jh = K.step(u, T, spec.L, g["dtau"], K.IMEX, 10)
        assert abs(Jh[0] - g["J_log"][i]) <= 1e-12 * abs(Jh[0])
    J = np.array(g["J_log"] + [g["J_final"]])
    assert np.all(np.diff(J) <= 0) and J[-1] < 2e-3 * J[0]
    assert np.all(np.abs(np.diff(g["T_log"])) < 1e-3)


# orbits the oracle reached from loops of its own chaotic runs, with the period the paper reports
ORBITS = [("oracle_orbit_L39.json", 25.37),  # Fig. 5a
          ("oracle_orbit_L39_T76.json", 76.61)]  # Fig. 5c


def _orbit_fixture(name="oracle_orbit_L39.json"):
    path = os.path.join(HERE, name)
    return json.load(open(path))


def _spectrum(modes, Nx, Ns):
    u = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    for j, k, re, im in modes:
        u[k % Ns, j] = complex(re, im)
    return u


@pytest.mark.parametrize("name,paper_T", ORBITS)
def test_oracle_orbit_is_a_papers_orbit(name, paper_T):
    """tests/golden/make_orbit.py cuts loops from the oracle's own chaotic runs at L = 39 and
    drives them with the oracle's loop dynamics (Sec. 4.3-4.4). Each stored converged loop is a
    periodic orbit by the oracle's own residual (J below the fixture's tolerance), and its period
    is one the paper reports: the shortest, T = 25.37 (Fig. 5a), and T = 76.61 (Fig. 5c), both
    to the paper's two decimals."""
    g = _orbit_fixture(name)
    u = _spectrum(g["uhat_final_band"], g["Nx"], g["Ns"])
    J = K.cost(u, g["T_final"], g["L"])
    assert J < g["J_tol"] and abs(J - g["J_final"]) <= 1e-6 * g["J_final"] + 1e-30
    assert abs(g["T_final"] - paper_T) < 0.005
    # it varies along s (not an equilibrium) and is centre-symmetric like its initial loop
    assert np.sum(np.abs(u[1:]) ** 2) > 1e-3 * np.sum(np.abs(u) ** 2)
    kneg = (-np.arange(g["Ns"])) % g["Ns"]
    assert np.max(np.abs(u + np.conj(u[kneg, :]))) < 1e-12 * np.max(np.abs(u))
