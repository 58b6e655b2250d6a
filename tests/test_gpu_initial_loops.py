"""GPU tests of the initial-loop pipeline (include/ks_initial_loops.h, Sec. 4.3) against the
oracle (oracle/ks_dns.py): the ETDRK4 runs (states, norms and samples to 1e-12, over runs
short enough that chaos has not amplified rounding), the recurrence pairs (exact: both sides
take the same IEEE comparisons on the same norm series), and the loops of segments (1e-13).
"""
import functools
import math

import numpy as np
import pytest

import loopgen
from oracle import ks_dns as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def il():
    from paper_2007_06427_amd import api, initial_loops
    torch.cuda.set_device(0)
    api.init()
    return initial_loops


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def runs(Nx, n, seed, scale, odd):
    rng = np.random.default_rng(seed)
    return np.stack([loopgen.random_ks_state(rng, Nx, scale=scale, odd=odd) for _ in range(n)])


@pytest.mark.parametrize("Nx,L", [(16, 22.0), (32, 22.0), (64, 39.0), (128, 39.0), (256, 100.0)])
@pytest.mark.parametrize("sym", [False, True])
def test_runs_match_oracle(il, Nx, L, sym):
    u0 = runs(Nx, 3, seed=Nx + sym, scale=0.8, odd=sym)
    if not sym:
        u0[:, 0] = 0.25  # a mean mode, carried unchanged
    dt, nsteps, every = 0.05, 60, 4
    u = torch.from_numpy(u0).to(DEV)
    ns = nsteps // every
    norms = torch.zeros(3, ns + 2, dtype=torch.float64, device=DEV)
    snaps = torch.zeros(3, ns + 2, Nx // 2 + 1, dtype=torch.complex128, device=DEV)
    il.ks_integrate(u, L, dt, nsteps, every, sym, norms, snaps, first_sample=1)
    ug, ng, sg = u.cpu().numpy(), norms.cpu().numpy(), snaps.cpu().numpy()
    for r in range(3):
        uo, no, so = D.integrate(u0[r], L, dt, nsteps, every, symmetric=sym)
        assert rel(ug[r], uo) < 1e-12, (Nx, sym, r)
        assert rel(ng[r, 1:ns + 1], no) < 1e-13
        assert rel(sg[r, 1:ns + 1], so) < 1e-12
        assert ng[r, 0] == 0 and ng[r, ns + 1] == 0  # nothing outside the samples of the call
        assert np.all(ug[r, (Nx - 1) // 3 + 1:] == 0)
        if sym:
            assert np.all(ug[r].real == 0)


def test_calls_chain(il):
    """Two calls of 40 steps give the one call of 80, bit for bit, samples included."""
    u0 = runs(64, 4, seed=1, scale=0.5, odd=True)
    a, b = torch.from_numpy(u0).to(DEV), torch.from_numpy(u0).to(DEV)
    na = torch.zeros(4, 20, dtype=torch.float64, device=DEV)
    sa = torch.zeros(4, 20, 33, dtype=torch.complex128, device=DEV)
    nb, sb = torch.zeros_like(na), torch.zeros_like(sa)
    il.ks_integrate(a, 39.0, 0.05, 80, 4, True, na, sa)
    il.ks_integrate(b, 39.0, 0.05, 40, 4, True, nb, sb)
    il.ks_integrate(b, 39.0, 0.05, 40, 4, True, nb, sb, first_sample=10)
    assert torch.equal(a, b) and torch.equal(na, nb) and torch.equal(sa, sb)


def test_out_of_band_mode_evolves_exactly(il):
    L, Nx, h, n = 39.0, 64, 0.05, 200
    K = (Nx - 1) // 3
    u0 = np.zeros((2, Nx // 2 + 1), dtype=np.complex128)
    u0[0, K] = 0.3 - 0.2j
    u0[1, K // 2 + 1] = 0.1j
    u = torch.from_numpy(u0).to(DEV)
    il.ks_integrate(u, L, h, n)
    ug = u.cpu().numpy()
    for r, j in ((0, K), (1, K // 2 + 1)):
        q = 2 * math.pi * j / L
        assert abs(ug[r, j] - math.exp((q * q - q ** 4) * n * h) * u0[r, j]) <= 1e-13 * abs(u0[r, j])


def test_chaotic_run_statistics_match_oracle(il):
    """A long centre-symmetric run at L = 39: trajectories separate (chaos), but the norm's
    range and mean agree with the oracle's run from the same start."""
    L, Nx, dt = 39.0, 64, 0.05
    u0 = runs(Nx, 1, seed=11, scale=0.1, odd=True)
    u = torch.from_numpy(u0).to(DEV)
    n = torch.zeros(1, 5000, dtype=torch.float64, device=DEV)
    il.ks_integrate(u, L, dt, 2000, 2000, True)
    il.ks_integrate(u, L, dt, 10000, 2, True, n)
    _, no, _ = D.integrate(D.integrate(u0[0], L, dt, 2000, symmetric=True)[0], L, dt, 10000, 2, symmetric=True)
    ng = n.cpu().numpy()[0]
    assert abs(ng.mean() - no.mean()) < 0.05 * no.mean()
    assert 6.0 < ng.min() and ng.max() < 11.0


@functools.lru_cache(maxsize=None)
def norm_series(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "ties":
        return np.round(rng.uniform(1.0, 2.0, size=3000), 2)
    L, Nx, dt = 39.0, 64, 0.05
    u, _, _ = D.integrate(loopgen.random_ks_state(rng, Nx, scale=0.1, odd=True), L, dt, 2000, 2000, symmetric=True)
    return D.integrate(u, L, dt, 16000, 2, symmetric=True)[1]


@pytest.mark.parametrize("kind,tol,Tmin,Tmax", [("ties", 0.02, 2.0, 9.0), ("ks", 0.01, 20.0, 160.0),
                                                ("ks", 0.002, 10.0, 300.0), ("ks", 0.0, 20.0, 160.0)])
def test_recurrences_equal_oracle(il, kind, tol, Tmin, Tmax):
    series = [norm_series(kind, s) for s in (1, 2, 3)]
    ns = len(series[0])
    dt_s = 0.1
    norms = torch.zeros(3, ns + 5, dtype=torch.float64, device=DEV)
    for r in range(3):
        norms[r, :ns] = torch.from_numpy(series[r])
    pairs, counts = il.ks_recurrences(norms, ns, dt_s, tol, Tmin, Tmax, cap=4096)
    pairs, counts = pairs.cpu().numpy(), counts.cpu().numpy()
    for r in range(3):
        want = D.recurrences(series[r], dt_s, tol, Tmin, Tmax)
        assert counts[r] == len(want)
        assert [tuple(p) for p in pairs[r, :counts[r]]] == want
    if tol == 0.0:
        assert counts.sum() < 3  # exact repeats of a chaotic norm are (almost) never seen


def test_recurrences_cap(il):
    s = norm_series("ties", 5)
    norms = torch.from_numpy(s[None]).to(DEV).contiguous()
    want = D.recurrences(s, 0.1, 0.02, 2.0, 9.0)
    pairs, counts = il.ks_recurrences(norms, len(s), 0.1, 0.02, 2.0, 9.0, cap=7)
    assert counts.item() == len(want) > 7
    assert [tuple(p) for p in pairs.cpu().numpy()[0]] == want[:7]


# (Nx, Ns, kc, L): 16 modes resolve the KS dynamics on L = 16 (on L = 39 the run blows up)
@pytest.mark.parametrize("Nx,Ns,kc,L", [(64, 64, 12, 39.0), (32, 128, 20, 39.0), (128, 32, 10, 39.0), (16, 8, 2, 16.0)])
def test_segments_match_oracle(il, Nx, Ns, kc, L):
    dt, every = 0.05, 2
    rng = np.random.default_rng(4 + Nx)
    u0 = np.stack([loopgen.random_ks_state(rng, Nx, scale=0.5, odd=o) for o in (True, False)])
    snaps_o = [D.integrate(u0[r], L, dt, 1200, every, symmetric=(r == 0))[2] for r in range(2)]
    assert all(np.all(np.isfinite(x)) for x in snaps_o)  # the oracle's runs are resolved
    ns = snaps_o[0].shape[0]
    snaps = torch.zeros(2, ns + 3, Nx // 2 + 1, dtype=torch.complex128, device=DEV)
    for r in range(2):
        snaps[r, :ns] = torch.from_numpy(snaps_o[r])
    dt_s = dt * every
    triples = [(0, 10, 290), (1, 0, 600), (1, 57, 100), (0, 3, 48), (1, 599, 600), (2, 0, 100), (0, 500, 601),
               (0, -1, 100), (1, 20, 40)]
    loops, T = il.ks_segments_to_loops(snaps, ns, torch.tensor(triples, dtype=torch.int32, device=DEV), dt_s, Ns, kc)
    loops, T = loops.cpu().numpy(), T.cpu().numpy()
    for l, (r, a, b) in enumerate(triples):
        if 0 <= r < 2 and 0 <= a and b <= ns and b - a > 2 * kc:
            uo, To = D.segment_to_loop(snaps_o[r], a, b, dt_s, Ns, kc)
            assert rel(loops[l], uo) < 1e-13, (r, a, b)
            assert T[l] == To
        else:  # invalid or too short: a zero loop and T = 0
            assert T[l] == 0 and np.all(loops[l] == 0), (r, a, b)


def test_pipeline_gives_centre_symmetric_loops(il):
    """The whole pipeline on 8 centre-symmetric runs: loops are invariant under Xi and their
    periods are those of the recurrences; each loop is the oracle's loop of its segment."""
    L, Nx, dt, every = 39.0, 64, 0.05, 2
    u0 = runs(Nx, 8, seed=9, scale=0.1, odd=True)
    u = torch.from_numpy(u0).to(DEV)
    loops, T, triples, norms, snaps = il.initial_loops(u, L, dt, 2000, 8000, every, 0.01, 20.0, 160.0, Ns=64, kc=10,
                                                       per_run=3)
    assert loops.shape[0] >= 8
    lo, Th, tr, sn = loops.cpu().numpy(), T.cpu().numpy(), triples.cpu().numpy(), snaps.cpu().numpy()
    kneg = (-np.arange(64)) % 64
    for l, (r, a, b) in enumerate(tr):
        assert 20.0 <= Th[l] <= 160.0 and Th[l] == (b - a) * (dt * every)
        assert np.max(np.abs(lo[l] + np.conj(lo[l][kneg, :]))) <= 1e-15 * np.max(np.abs(lo[l]))
        uo, To = D.segment_to_loop(sn[r], a, b, dt * every, 64, 10)
        assert rel(lo[l], uo) < 1e-13


def test_binding_rejects_bad_arguments(il):
    from paper_2007_06427_amd import LoopOrbitError
    u = torch.zeros(2, 33, dtype=torch.complex128, device=DEV)
    n = torch.zeros(2, 10, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):  # a CPU tensor
        il.ks_integrate(torch.zeros(2, 33, dtype=torch.complex128), 39.0, 0.05, 8)
    with pytest.raises(ValueError):  # the samples of the call do not fit after first_sample
        il.ks_integrate(u, 39.0, 0.05, 40, 4, norms=n, first_sample=1)
    with pytest.raises(ValueError):  # one row per run
        il.ks_integrate(u, 39.0, 0.05, 8, 4, norms=torch.zeros(3, 10, dtype=torch.float64, device=DEV))
    with pytest.raises(LoopOrbitError):  # 512-point runs are not compiled in
        il.ks_integrate(torch.zeros(1, 257, dtype=torch.complex128, device=DEV), 39.0, 0.05, 8)
    with pytest.raises(LoopOrbitError):  # sample_every does not divide nsteps
        il.ks_integrate(u, 39.0, 0.05, 10, 4)
    with pytest.raises(LoopOrbitError):  # kc beyond the loop band
        il.ks_segments_to_loops(torch.zeros(1, 10, 33, dtype=torch.complex128, device=DEV), 10,
                                torch.zeros(1, 3, dtype=torch.int32, device=DEV), 0.1, 16, 6)
    assert torch.equal(u, torch.zeros_like(u))  # nothing ran
