"""GPU tests of the LDS-resident form of loop_step (one block per loop, all steps in one launch).

Its column passes are the per-pass form's own bodies and its row passes pair rows the same
way, so each step must equal the per-pass batch form bit for bit (J history, T and the
spectrum), and match the oracle to 1e-12 per step (normwise, as in test_gpu_parity.py).
"""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# shapes the resident form takes: both ends of the size range, the workloads' 32 x 32 and
# 64 x 128, and the largest working sets (about 155 KB of LDS)
SHAPES = [(8, 8), (8, 512), (16, 256), (32, 32), (32, 256), (64, 64), (64, 128), (128, 8), (128, 64)]


@pytest.fixture(scope="module")
def api():
    from paper_2007_06427_amd import api as A
    torch.cuda.set_device(0)
    A.init()
    prev = A.set_resident(A.RESIDENT_ALWAYS)
    yield A
    A.set_resident(prev)


def wrel(a, b):
    w = np.full(a.shape[-1], 2.0)
    w[0] = 1.0
    return np.sqrt(np.sum(w * np.abs(a - b) ** 2)) / max(np.sqrt(np.sum(w * np.abs(b) ** 2)), 1e-300)


def loops(Nx, Ns, n, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    u = np.stack([loopgen.random_band_field(rng, Nx, Ns, scale=scale) for _ in range(n)])
    T = rng.uniform(20.0, 80.0, size=n)
    return u, T


def resident_step(api, u, T, L, dtau, scheme, nsteps):
    ud = torch.from_numpy(u).to(DEV)
    Td = torch.tensor(T, dtype=torch.float64, device=DEV)
    Jh = torch.zeros(max(nsteps, 1), len(T), dtype=torch.float64, device=DEV)
    ws = api.Workspace(api.workspace_bytes((u.shape[2] - 1) * 2, u.shape[1], len(T)))
    api.loop_step(ud, Td, L, dtau, scheme, nsteps, J_hist=Jh, ws=ws)
    torch.cuda.synchronize()
    assert ws.status() == 0
    return ud.cpu().numpy(), Td.cpu().numpy(), Jh.cpu().numpy()


def batch_step(api, u, T, L, dtau, scheme, nsteps):
    Ns, H = u.shape[1], u.shape[2]
    Nx = (H - 1) * 2
    b = api.Batch([(L, Nx, Ns)] * len(T))
    b.set_schedule(api.Batch.PER_PASS)
    pool = b.pack([torch.from_numpy(x) for x in u])
    Td = torch.tensor(T, dtype=torch.float64, device=DEV)
    Jh = torch.zeros(max(nsteps, 1), len(T), dtype=torch.float64, device=DEV)
    b.step(pool, Td, dtau, scheme, nsteps, J_hist=Jh)
    torch.cuda.synchronize()
    assert b.status() == 0
    return np.stack([x.cpu().numpy() for x in b.unpack(pool)]), Td.cpu().numpy(), Jh.cpu().numpy()


def test_supported_shapes(api):
    for Nx, Ns in SHAPES:
        assert api.resident_supported(Nx, Ns), (Nx, Ns)
    for Nx, Ns in [(64, 256), (32, 512), (256, 64), (128, 128), (8, 1024), (1024, 8)]:
        assert not api.resident_supported(Nx, Ns), (Nx, Ns)
    assert not api.resident_supported(48, 32)


@pytest.mark.parametrize("Nx,Ns", SHAPES)
@pytest.mark.parametrize("scheme", [0, 1])
def test_resident_equals_per_pass_bitwise(api, Nx, Ns, scheme):
    u, T = loops(Nx, Ns, 3, seed=Nx * 1000 + Ns)
    L = 22.0 if Nx <= 32 else 39.0
    dtau = 1e-5 if scheme == 1 else 1e-7  # explicit: inside the stability limit of every shape here
    a = resident_step(api, u, T, L, dtau, scheme, 4)
    b = batch_step(api, u, T, L, dtau, scheme, 4)
    assert np.array_equal(a[2][:4], b[2][:4]), (Nx, Ns)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("Nx,Ns", SHAPES)
def test_resident_one_step_matches_oracle(api, Nx, Ns):
    u, T = loops(Nx, Ns, 2, seed=7 + Nx + Ns)
    L = 22.0
    ug, Tg, Jg = resident_step(api, u, T, L, 5e-5, 1, 1)
    for i in range(2):
        uo, To, Jo = K.step(u[i], T[i], L, 5e-5, K.IMEX, 1)
        assert wrel(ug[i], uo) < 1e-12, (Nx, Ns)
        assert abs(Tg[i] - To) <= 1e-12 * abs(To)
        assert abs(Jg[0, i] - Jo[0]) <= 1e-12 * Jo[0]


def test_resident_equals_per_pass_loop_step(api):
    """Mode 0 routes loop_step to the per-pass kernels; with one loop (rows are paired within
    the loop on both paths) the results agree bit for bit."""
    u, T = loops(64, 128, 1, seed=3)
    a = resident_step(api, u, T, 22.0, 5e-5, 1, 6)
    prev = api.set_resident(api.RESIDENT_NEVER)
    try:
        assert prev == api.RESIDENT_ALWAYS
        b = resident_step(api, u, T, 22.0, 5e-5, 1, 6)
    finally:
        api.set_resident(prev)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_zero_steps_canonicalises(api):
    rng = np.random.default_rng(4)
    u = np.stack([rng.standard_normal((32, 17)) + 1j * rng.standard_normal((32, 17)) for _ in range(2)])
    T = np.array([30.0, 40.0])
    ug, Tg, _ = resident_step(api, u, T, 22.0, 1e-4, 0, 0)
    for i in range(2):
        assert np.abs(ug[i] - K.canonical(u[i])).max() < 1e-16
    assert np.array_equal(Tg, T)


def test_many_loops_one_launch(api):
    """512 loops of 32 x 64: two loops per CU at once, each block independent."""
    u, T = loops(32, 64, 512, seed=11, scale=0.2)
    ug, Tg, Jg = resident_step(api, u, T, 22.0, 5e-5, 1, 3)
    for i in (0, 255, 511):
        uo, To, Jo = K.step(u[i], T[i], 22.0, 5e-5, K.IMEX, 3)
        assert wrel(ug[i], uo) < 1e-12
        assert abs(Tg[i] - To) <= 1e-12 * abs(To)
        assert np.allclose(Jg[:, i], Jo, rtol=1e-12, atol=0)


def test_resident_flags_nonpositive_period(api):
    from paper_2007_06427_amd import _lib
    u, T = loops(32, 32, 2, seed=5)
    T[1] = -1.0
    ud = torch.from_numpy(u).to(DEV)
    Td = torch.tensor(T, dtype=torch.float64, device=DEV)
    ws = api.Workspace(api.workspace_bytes(32, 32, 2))
    api.loop_step(ud, Td, 22.0, 1e-4, 1, 2, ws=ws)
    assert ws.status() == _lib.LOOP_ENONFINITE


def test_set_resident_rejects_other_values(api):
    from paper_2007_06427_amd import _lib
    assert _lib.lib().loop_set_resident(3) == _lib.LOOP_EINVAL
    assert _lib.lib().loop_set_resident(-1) == _lib.LOOP_EINVAL


def test_auto_mode_gives_the_same_results(api):
    """Whichever form the automatic choice takes, loop_step's results are those of the
    resident form (one loop: identical bits)."""
    for (Nx, Ns) in [(32, 32), (64, 128)]:
        u, T = loops(Nx, Ns, 1, seed=Nx + Ns)
        a = resident_step(api, u, T, 22.0, 5e-5, 1, 3)
        prev = api.set_resident(api.RESIDENT_AUTO)
        try:
            b = resident_step(api, u, T, 22.0, 5e-5, 1, 3)
        finally:
            api.set_resident(prev)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
