"""GPU tests of the batched form: loops of uneven (L, Nx, Ns) in one persistent launch.

Parity bar: 1e-12 relative per step against the CPU oracle (normwise, as in
test_gpu_parity.py). The batched kernel runs the same pass code as loop_step, so each loop
must also match loop_step on that loop alone, bit for bit.
"""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    from paper_2007_06427_amd import api as A
    torch.cuda.set_device(0)
    A.init()
    return A


def wrel(a, b):
    w = np.full(a.shape[-1], 2.0)
    w[0] = 1.0
    return np.sqrt(np.sum(w * np.abs(a - b) ** 2)) / max(np.sqrt(np.sum(w * np.abs(b) ** 2)), 1e-300)


def ragged_specs(n, seed=7):
    """n loops drawn like the ragged workload: Nx in {32, 64}, Ns in {64..512}, L in {22, 39},
    plus a few odd shapes at the edges (8 x 1024, 512 x 16, 16 x 8)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        Nx = int(rng.choice([32, 64]))
        Ns = int(rng.choice([64, 128, 256, 512]))
        L = float(rng.choice([22.0, 39.0]))
        T = float(rng.uniform(20.0, 80.0))
        u = loopgen.seeded_spectrum(rng, Nx, Ns, 4, 3, 0.5, 0.3)
        out.append((L, Nx, Ns, T, u))
    for (Nx, Ns, L) in [(8, 1024, 7.0), (512, 16, 150.0), (16, 8, 9.0)]:
        T = float(rng.uniform(20.0, 80.0))
        out.append((L, Nx, Ns, T, loopgen.random_band_field(rng, Nx, Ns, scale=0.2)))
    return out


SCHEDULES = [0, 1, 2]  # per-pass launches, persistent, two streams


def run_batch(api, specs, nsteps, dtau, scheme, schedule=0, nstreams=2):
    b = api.Batch([(L, Nx, Ns) for (L, Nx, Ns, T, u) in specs])
    b.set_schedule(schedule, nstreams)
    pool = b.pack([torch.from_numpy(u) for (*_, u) in specs])
    T = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    Jh = torch.zeros(max(nsteps, 1), len(specs), dtype=torch.float64, device=DEV)
    b.step(pool, T, dtau, scheme, nsteps, J_hist=Jh)
    torch.cuda.synchronize()
    assert b.status() == 0
    return b, [x.cpu().numpy() for x in b.unpack(pool)], T.cpu().numpy(), Jh.cpu().numpy()


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_batch_matches_single_loop_steps_bitwise(api, schedule):
    specs = ragged_specs(13)
    _, ub, Tb, Jb = run_batch(api, specs, 5, 5e-5, api.IMEX, schedule)
    for i, (L, Nx, Ns, T0, u0) in enumerate(specs):
        u = torch.from_numpy(u0[None]).to(DEV)
        T = torch.tensor([T0], dtype=torch.float64, device=DEV)
        Jh = torch.zeros(5, 1, dtype=torch.float64, device=DEV)
        api.loop_step(u, T, L, 5e-5, api.IMEX, 5, J_hist=Jh)
        assert np.array_equal(u.cpu().numpy()[0], ub[i]), (i, Nx, Ns)
        assert T.item() == Tb[i]
        assert np.array_equal(Jh.cpu().numpy()[:, 0], Jb[:, i])


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("scheme", [0, 1])
def test_batch_matches_oracle(api, scheme, schedule):
    """One step and three steps from identical inputs on every loop of a ragged batch: six
    low-mode loops and three full-band stress fields (8 x 1024, 512 x 16, 16 x 8). The oracle
    is well conditioned here: three of its FP64 steps agree with the same steps in long double
    to 6e-16 on every loop, and the device's three steps measured within 9e-16 of the oracle."""
    specs = ragged_specs(6, seed=11)
    dtau = 5e-5
    if scheme == 0:  # explicit Euler: stay inside its stability limit dtau < 2 / |lambda|max
        lam_max = max(np.abs(K.lam(T, L, Nx, Ns)[K.band_mask(Nx, Ns)]).max() for (L, Nx, Ns, T, u) in specs)
        dtau = 0.5 / lam_max
    for nsteps, subset in ((1, specs), (3, specs)):
        _, ub, Tb, Jb = run_batch(api, subset, nsteps, dtau, scheme, schedule)
        for i, (L, Nx, Ns, T0, u0) in enumerate(subset):
            uo, To, Jo = K.step(u0, T0, L, dtau, scheme, nsteps)
            assert wrel(ub[i], uo) < 1e-12, (nsteps, i, Nx, Ns, wrel(ub[i], uo))
            assert abs(Tb[i] - To) <= 1e-12 * To
            assert np.all(np.abs(Jb[:nsteps, i] - Jo) <= 1e-12 * Jo)


def test_persistent_wait_that_runs_out_is_reported_and_the_next_launch_is_clean(api):
    """A dependency wait of the persistent schedule that runs out abandons the launch: with a
    wait bound of zero the first wait that does not succeed at once does so, every block leaves
    at its next wait, and the status says LOOP_EHANG. The next launch on the same work space,
    with the default bound, clears the schedule's counters first and equals the per-pass
    schedule bit for bit."""
    from paper_2007_06427_amd import _lib
    specs = ragged_specs(8, seed=21)
    ref = run_batch(api, specs, 3, 5e-5, api.IMEX, 0)
    b = api.Batch([(L, Nx, Ns) for (L, Nx, Ns, T, u) in specs])
    b.set_schedule(api.Batch.PERSISTENT)
    pool0 = b.pack([torch.from_numpy(u) for (*_, u) in specs])
    T0 = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    b.set_wait_limit(0.0)
    pool, T = pool0.clone(), T0.clone()
    b.step(pool, T, 5e-5, api.IMEX, 3)
    torch.cuda.synchronize()
    assert b.status() == _lib.LOOP_EHANG
    b.set_wait_limit(2.0)
    for _ in range(2):
        pool, T = pool0.clone(), T0.clone()
        Jh = torch.zeros(3, len(specs), dtype=torch.float64, device=DEV)
        b.step(pool, T, 5e-5, api.IMEX, 3, J_hist=Jh)
        torch.cuda.synchronize()
        assert b.status() == 0
        for i, u in enumerate(b.unpack(pool)):
            assert np.array_equal(u.cpu().numpy(), ref[1][i])
        assert np.array_equal(T.cpu().numpy(), ref[2]) and np.array_equal(Jh.cpu().numpy(), ref[3])


@pytest.mark.parametrize("n", [1, 5, 11, 40])
def test_persistent_schedule_equals_per_pass_for_any_number_of_loops(api, n):
    """The persistent schedule gives each loop to one XCD and hands tiles over only inside that
    XCD's L2; with fewer loops than XCDs some XCDs' lists are empty. Ten steps of n loops (the
    edge shapes 8 x 1024, 512 x 16 and 16 x 8 among them) equal the per-pass schedule bit for
    bit, periods and J history included."""
    specs = ragged_specs(max(n - 3, 0), seed=40 + n)[:n]
    _, u0, T0, J0 = run_batch(api, specs, 10, 5e-5, api.IMEX, 0)
    b, u1, T1, J1 = run_batch(api, specs, 10, 5e-5, api.IMEX, 1)
    assert b.status() == 0
    assert all(np.array_equal(a, c) for a, c in zip(u0, u1))
    assert np.array_equal(T0, T1) and np.array_equal(J0, J1)


def test_persistent_schedule_over_many_steps_and_launches(api):
    """Sixty steps of 48 loops in one launch, twice, each equal to the per-pass schedule bit for
    bit: a tile read before its producer's stores were in the L2 its consumer reads would show
    here."""
    specs = ragged_specs(45, seed=5)
    _, u0, T0, J0 = run_batch(api, specs, 60, 5e-5, api.IMEX, 0)
    b = api.Batch([(L, Nx, Ns) for (L, Nx, Ns, T, u) in specs])
    b.set_schedule(api.Batch.PERSISTENT)
    pool0 = b.pack([torch.from_numpy(u) for (*_, u) in specs])
    Tin = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    for _ in range(2):
        pool, T = pool0.clone(), Tin.clone()
        Jh = torch.zeros(60, len(specs), dtype=torch.float64, device=DEV)
        b.step(pool, T, 5e-5, api.IMEX, 60, J_hist=Jh)
        torch.cuda.synchronize()
        assert b.status() == 0
        assert all(np.array_equal(u.cpu().numpy(), w) for u, w in zip(b.unpack(pool), u0))
        assert np.array_equal(T.cpu().numpy(), T0) and np.array_equal(Jh.cpu().numpy(), J0)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_batch_zero_steps_canonicalises_and_relaunches(api, schedule):
    specs = ragged_specs(4, seed=3)
    b, ub, Tb, _ = run_batch(api, specs, 0, 1e-4, api.EXPLICIT, schedule)
    for i, (L, Nx, Ns, T0, u0) in enumerate(specs):
        assert np.abs(ub[i] - K.canonical(u0)).max() < 1e-16
        assert Tb[i] == T0
    # the same plan and work space serve several launches in a row
    pool = b.pack([torch.from_numpy(u) for (*_, u) in specs])
    T = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    for _ in range(3):
        b.step(pool, T, 5e-5, api.IMEX, 2)
    torch.cuda.synchronize()
    assert b.status() == 0
    u1 = [x.cpu().numpy() for x in b.unpack(pool)]
    for i, (L, Nx, Ns, T0, u0) in enumerate(specs):
        uo, To, _ = K.step(u0, T0, L, 5e-5, K.IMEX, 6)
        assert wrel(u1[i], uo) < 1e-12


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_batch_graph_replay_matches_eager(api, schedule):
    specs = ragged_specs(8, seed=5)
    b = api.Batch([(L, Nx, Ns) for (L, Nx, Ns, T, u) in specs])
    b.set_schedule(schedule)
    u0 = [torch.from_numpy(u) for (*_, u) in specs]
    T0 = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    # eager reference: 4 launches of 2 steps
    pe = b.pack(u0)
    Te = T0.clone()
    for _ in range(4):
        b.step(pe, Te, 5e-5, api.IMEX, 2)
    # graph: capture one launch of 2 steps, replay 4 times with eager work in between
    pg = b.pack(u0)
    Tg = T0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.step(pg.clone(), Tg.clone(), 5e-5, api.IMEX, 1)  # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    b.reset()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.step(pg, Tg, 5e-5, api.IMEX, 2)
    for k in range(4):
        g.replay()
        torch.cuda.synchronize()
        _ = (pg.abs().sum()).item()  # unrelated eager work between replays
    assert b.status() == 0
    assert torch.equal(pg, pe) and torch.equal(Tg, Te)


def test_batch_rejects_bad_plans(api):
    from paper_2007_06427_amd import _lib
    with pytest.raises(_lib.LoopOrbitError):
        api.Batch([(22.0, 48, 64)])
    with pytest.raises(_lib.LoopOrbitError):
        api.Batch([(22.0, 1024, 64)])  # batched row passes take Nx <= 512
    with pytest.raises(_lib.LoopOrbitError):
        api.Batch([(-1.0, 32, 64)])


def test_pass_building_blocks_equal_batch_step(api):
    specs = ragged_specs(9, seed=21)
    nsteps = 3
    b, ub, Tb, Jb = run_batch(api, specs, nsteps, 5e-5, api.IMEX)
    pool = b.pack([torch.from_numpy(u) for (*_, u) in specs])
    T = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    Jh = torch.zeros(nsteps, len(specs), dtype=torch.float64, device=DEV)
    b.load(pool)
    b.run_pass(0, 0, nsteps, T, 5e-5, api.IMEX, Jh)
    for s in range(nsteps):
        for p in (1, 2, 3, 4):
            b.run_pass(p, s, nsteps, T, 5e-5, api.IMEX, Jh)
    b.store(pool)
    torch.cuda.synchronize()
    assert b.status() == 0
    for i, x in enumerate(b.unpack(pool)):
        assert np.array_equal(x.cpu().numpy(), ub[i])
    assert np.array_equal(T.cpu().numpy(), Tb) and np.array_equal(Jh.cpu().numpy(), Jb)


@pytest.mark.parametrize("n", [1, 2, 5, 13])
@pytest.mark.parametrize("nstreams", [2, 3, 4])
def test_stream_schedule_equals_per_pass(api, n, nstreams):
    """The multi-stream schedule with one loop (its other groups are empty) up to thirteen,
    over 1 and 4 steps, against the per-pass schedule bit for bit."""
    specs = ragged_specs(n, seed=21)[:n]
    for nsteps in (1, 4):
        _, ua, Ta, Ja = run_batch(api, specs, nsteps, 5e-5, api.IMEX, 0)
        _, ub, Tb, Jb = run_batch(api, specs, nsteps, 5e-5, api.IMEX, 2, nstreams)
        for x, y in zip(ua, ub):
            assert np.array_equal(x, y)
        assert np.array_equal(Ta, Tb) and np.array_equal(Ja, Jb)


def test_set_streams_rejects_counts_outside_2_to_4(api):
    b = api.Batch([(22.0, 32, 64)])
    for k in (1, 5):
        with pytest.raises(api.LoopOrbitError):
            b.set_schedule(2, k)
