"""GPU tests of the convergence driver loop_converge (Sec. 4.3, App. C) against the oracle's
driver (oracle/accelerate.py), whose runs from the 32 x 32 workload's seed are stored in
tests/golden/oracle_accelerated_plain32x32.json (written by tests/golden/make_golden.py).

Both drivers examine J after every `stride` steps and take their decisions from it, so the
GPU run must take the same number of steps and extrapolations as the oracle's, and end on
the same state: T to 1e-8 and band-mode magnitudes to 1e-8.
"""
import json
import os

import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def api():
    from paper_2007_06427_amd import api as A
    torch.cuda.set_device(0)
    A.init()
    return A


@pytest.fixture(scope="module")
def golden():
    return json.load(open(os.path.join(HERE, "oracle_accelerated_plain32x32.json")))


@pytest.mark.parametrize("accelerate", [False, True])
@pytest.mark.parametrize("form", [0, 2])  # loop_step per-pass, LDS-resident
def test_driver_matches_oracle_driver(api, golden, accelerate, form):
    run = golden["runs"][1 if accelerate else 0]
    assert run["accelerate"] == accelerate
    spec = loopgen.config_loops(1)[0]
    u = torch.from_numpy(spec.uhat[None]).to(DEV)
    T = torch.tensor([spec.T], dtype=torch.float64, device=DEV)
    prev = api.set_resident(form)
    try:
        res = api.loop_converge(u, T, spec.L, golden["dtau"], K.IMEX, golden["J_tol"], stride=golden["stride"],
                                accelerate=accelerate, sqrtJ_first=golden["sqrtJ_first"])
    finally:
        api.set_resident(prev)
    assert res["steps"][0] == run["steps"]
    assert res["extrapolations"][0] == run["extrapolations"]
    assert res["J"][0] < golden["J_tol"]
    assert abs(res["J"][0] - run["J_final"]) <= 1e-3 * run["J_final"]
    assert abs(T.item() - run["T_final"]) <= 1e-8
    ug = u.cpu().numpy()[0]
    worst = max(abs(abs(ug[k % spec.Ns, j]) - a) for j, k, a in run["abs_uhat_final_band"])
    assert worst <= 1e-8, worst
    # the returned state is the one the driver stopped on
    assert abs(api.loop_cost(u, T, spec.L).item() - res["J"][0]) <= 1e-12 * res["J"][0]


def test_acceleration_saves_steps(golden):
    plain, acc = golden["runs"]
    assert acc["extrapolations"] >= 1
    assert acc["steps"] < 0.7 * plain["steps"]


def test_batch_equals_single_loop_runs(api):
    """Three loops driven together: each converges after the steps it needs alone, with the
    same extrapolations, and keeps the state at which it converged."""
    specs = [loopgen.random_loop(s, 14.0, 16, 16, 2, 2, 0.8, 0.3, 20.0) for s in (5, 7, 8)]
    L = specs[0].L
    alone = []
    for s in specs:
        u = torch.from_numpy(s.uhat[None]).to(DEV)
        T = torch.tensor([s.T], dtype=torch.float64, device=DEV)
        r = api.loop_converge(u, T, L, 0.1, K.IMEX, 1e-10, stride=20, max_steps=60000, accelerate=True)
        alone.append((r, u.cpu().numpy()[0], T.item()))
    u = torch.from_numpy(np.stack([s.uhat for s in specs])).to(DEV)
    T = torch.tensor([s.T for s in specs], dtype=torch.float64, device=DEV)
    rb = api.loop_converge(u, T, L, 0.1, K.IMEX, 1e-10, stride=20, max_steps=60000, accelerate=True)
    ub, Tb = u.cpu().numpy(), T.cpu().numpy()
    assert len(set(rb["steps"])) > 1  # the loops converge at different times
    for i, (r, ui, Ti) in enumerate(alone):
        assert r["steps"][0] > 0
        assert rb["steps"][i] == r["steps"][0] and rb["extrapolations"][i] == r["extrapolations"][0]
        assert np.abs(ub[i] - ui).max() <= 1e-12 * np.abs(ui).max()
        assert abs(Tb[i] - Ti) <= 1e-12 * Ti


def test_not_converged_within_max_steps(api):
    spec = loopgen.config_loops(1)[0]
    u = torch.from_numpy(spec.uhat[None]).to(DEV)
    T = torch.tensor([spec.T], dtype=torch.float64, device=DEV)
    r = api.loop_converge(u, T, spec.L, 0.05, K.IMEX, 1e-10, stride=100, max_steps=1000, accelerate=True)
    assert r["steps"] == [-1]
    assert r["J"][0] > 1e-10
    assert abs(api.loop_cost(u, T, spec.L).item() - r["J"][0]) <= 1e-12 * r["J"][0]


def test_rejects_bad_arguments(api):
    spec = loopgen.config_loops(1)[0]
    u = torch.from_numpy(spec.uhat[None]).to(DEV)
    T = torch.tensor([spec.T], dtype=torch.float64, device=DEV)
    for kw in ({"stride": 0}, {"J_tol": 0.0}, {"J_tol": -1.0}, {"sqrtJ_first": 0.0}, {"max_steps": -1}):
        args = {"stride": 10, "J_tol": 1e-10, "sqrtJ_first": 1e-3, "max_steps": 10}
        args.update(kw)
        with pytest.raises(api.LoopOrbitError):
            api.loop_converge(u, T, spec.L, 0.05, K.IMEX, args["J_tol"], stride=args["stride"],
                              max_steps=args["max_steps"], sqrtJ_first=args["sqrtJ_first"])
