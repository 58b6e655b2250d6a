"""GPU tests of the kernel variants and the autotuner of the batched per-pass schedule.

Variants 0-2 of a pass run the same arithmetic on the same tiles, so a step taken with any of
them must equal the all-variant-0 step bit for bit, and that step must match the oracle to
1e-12 (normwise, per loop, as in test_gpu_parity.py). Row variant 3 (four points per thread)
pairs rows and factors its transforms differently: it must meet the same 1e-12 bound against
the oracle. The autotuner must leave the caller's
state untouched, choose the fastest candidate it timed, and hand its choice to later plans of
the same shapes.
"""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PASSES = range(5)


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


def specs_from(shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for (Nx, Ns) in shapes:
        L = float(rng.choice([22.0, 39.0]))
        T = float(rng.uniform(20.0, 80.0))
        out.append((L, Nx, Ns, T, loopgen.random_band_field(rng, Nx, Ns, scale=0.3)))
    return out


# every variant of every pass covers these sizes (Nx and Ns up to 64)
SMALL = [(Nx, Ns) for Nx in (8, 16, 32, 64) for Ns in (8, 16, 32, 64)]
# the ragged workload's sizes: row variants 0, 1, 2 and column variants 0, 2 cover them
RAGGED = [(Nx, Ns) for Nx in (32, 64) for Ns in (64, 128, 256, 512)] * 2
# sizes only variant 0 covers, for rows (Nx = 128) and for columns (Ns = 1024)
LARGE = [(128, 64), (32, 1024), (64, 128)]


def usable(api, batch):
    """(pass, variant) pairs the plan accepts; the plan's own choice is restored after."""
    keep = batch.config()["variants"]
    out = []
    for p in PASSES:
        for v in range(api.Batch.VARIANTS):
            try:
                batch.set_variant(p, v)
                out.append((p, v))
            except api.LoopOrbitError:
                pass
        batch.set_variant(p, keep[api.Batch.PASS_NAMES[p]])
    return out


def step_with(api, batch, specs, variants, nsteps=3):
    for p, v in variants.items():
        batch.set_variant(p, v)
    batch.set_schedule(api.Batch.PER_PASS)
    pool = batch.pack([torch.from_numpy(s[4]) for s in specs])
    T = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    Jh = torch.zeros(nsteps, len(specs), dtype=torch.float64, device=DEV)
    batch.step(pool, T, 5e-5, api.IMEX, nsteps, J_hist=Jh)
    torch.cuda.synchronize()
    assert batch.status() == 0
    return pool.cpu().numpy(), T.cpu().numpy(), Jh.cpu().numpy()


@pytest.mark.parametrize("name,shapes", [("small", SMALL), ("ragged", RAGGED), ("large", LARGE)])
def test_every_variant_equals_variant0_bitwise(api, name, shapes):
    specs = specs_from(shapes, 11)
    b = api.Batch([(s[0], s[1], s[2]) for s in specs])
    ok = usable(api, b)
    expect = {"small": 17, "ragged": 14, "large": 5}[name]
    assert len(ok) == expect, ok
    ok = [(p, v) for (p, v) in ok if v < 3]  # row variant 3 agrees to rounding only
    base = step_with(api, b, specs, {p: 0 for p in PASSES})
    for (p, v) in ok:
        if v == 0:
            continue
        got = step_with(api, b, specs, {**{q: 0 for q in PASSES}, p: v})
        for x, y in zip(got, base):
            assert np.array_equal(x, y), (name, p, v)
    # every pass on its last usable variant at once (the DMA row loader where usable)
    last = {p: max(v for (q, v) in ok if q == p) for p in PASSES}
    got = step_with(api, b, specs, last)
    for x, y in zip(got, base):
        assert np.array_equal(x, y), (name, last)


def test_variant0_step_matches_oracle(api):
    specs = specs_from(SMALL[::3] + RAGGED[:8], 12)
    b = api.Batch([(s[0], s[1], s[2]) for s in specs])
    pool, T, _ = step_with(api, b, specs, {p: 0 for p in PASSES}, nsteps=1)
    for i, (L, Nx, Ns, T0, u0) in enumerate(specs):
        uo, To, _ = K.step(u0, T0, L, 5e-5, K.IMEX, 1)
        off = b.offsets[i]
        ug = pool[off:off + Ns * (Nx // 2 + 1)].reshape(Ns, Nx // 2 + 1)
        assert wrel(ug, uo) < 1e-12, (Nx, Ns)
        assert abs(T[i] - To) <= 1e-12 * abs(To)


@pytest.mark.parametrize("name,shapes", [("small", SMALL), ("ragged", RAGGED)])
def test_row_variant3_matches_oracle(api, name, shapes):
    specs = specs_from(shapes[::2], 15)
    b = api.Batch([(s[0], s[1], s[2]) for s in specs])
    pool, T, Jh = step_with(api, b, specs, {1: 3, 3: 3}, nsteps=2)
    for i, (L, Nx, Ns, T0, u0) in enumerate(specs):
        uo, To, Jo = K.step(u0, T0, L, 5e-5, K.IMEX, 2)
        off = b.offsets[i]
        ug = pool[off:off + Ns * (Nx // 2 + 1)].reshape(Ns, Nx // 2 + 1)
        assert wrel(ug, uo) < 1e-12, (Nx, Ns)
        assert abs(T[i] - To) <= 1e-12 * abs(To)
        assert np.allclose(Jh[:, i], Jo, rtol=1e-12, atol=0)


def test_set_variant_rejects_sizes_it_does_not_cover(api):
    b = api.Batch([(22.0, 128, 64), (22.0, 32, 1024)])
    for v in (1, 2, 3):
        for p in (1, 3):  # row passes: Nx = 128 is beyond 64
            with pytest.raises(api.LoopOrbitError):
                b.set_variant(p, v)
        for p in (0, 2, 4):  # column passes: Ns = 1024 is beyond 512
            with pytest.raises(api.LoopOrbitError):
                b.set_variant(p, v)
    for bad in (-1, 4):
        with pytest.raises(api.LoopOrbitError):
            b.set_variant(1, bad)
    b2 = api.Batch([(22.0, 32, 64)])
    b2.set_variant(1, 3)  # row passes have a fourth variant, column passes do not
    with pytest.raises(api.LoopOrbitError):
        b2.set_variant(2, 3)
    with pytest.raises(api.LoopOrbitError):
        b.set_variant(5, 0)


def test_autotune_keeps_state_picks_fastest_and_is_reused(api):
    specs = specs_from(RAGGED, 13)
    shapes = [(s[0], s[1], s[2]) for s in specs]
    b = api.Batch(shapes)
    pool = b.pack([torch.from_numpy(s[4]) for s in specs])
    T = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    p0, T0 = pool.clone(), T.clone()
    rep = b.autotune(pool, T, reps=5)
    torch.cuda.synchronize()
    assert torch.equal(pool, p0) and torch.equal(T, T0)
    assert b.status() == 0
    for name, times in rep["pass_us"].items():
        assert len(times) >= 1 and all(t > 0 for t in times.values())
        # the plan's variant stays unless another is faster by more than 1% (times rounded to ns)
        assert 0.99 * times[rep["variants"][name]] <= min(times.values()) + 1e-3, (name, rep)
    su = rep["step_us"]
    assert set(su) == {"per-pass", "streams-2", "streams-3", "streams-4"}  # persistent: not timed
    assert all(v > 0 for v in su.values())
    assert su[rep["schedule"]] == min(su.values())
    # a later plan with the same multiset of shapes (in another order) starts from the choice
    b2 = api.Batch(shapes[::-1])
    assert b2.config() == {"schedule": rep["schedule"], "variants": rep["variants"]}
    # and the tuned configuration steps exactly like variant 0 on the per-pass schedule
    base = step_with(api, api.Batch(shapes), specs, {p: 0 for p in PASSES})
    pool2, T2 = p0.clone(), T0.clone()
    Jh = torch.zeros(3, len(specs), dtype=torch.float64, device=DEV)
    b.step(pool2, T2, 5e-5, api.IMEX, 3, J_hist=Jh)
    torch.cuda.synchronize()
    assert b.status() == 0
    assert np.array_equal(pool2.cpu().numpy(), base[0])
    assert np.array_equal(T2.cpu().numpy(), base[1])
    assert np.array_equal(Jh.cpu().numpy(), base[2])


def test_autotune_rejects_bad_arguments(api):
    specs = specs_from(SMALL[:4], 14)
    b = api.Batch([(s[0], s[1], s[2]) for s in specs])
    pool = b.pack([torch.from_numpy(s[4]) for s in specs])
    T = torch.tensor([s[3] for s in specs], dtype=torch.float64, device=DEV)
    for reps in (0, 1001):
        with pytest.raises(api.LoopOrbitError):
            b.autotune(pool, T, reps=reps)
    with pytest.raises(ValueError):
        b.autotune(pool[:-1], T)
