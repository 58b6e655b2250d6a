"""Every stepping entry point can be recorded into a HIP graph (no call synchronises, allocates
or records a memset): one captured call replayed three times, with unrelated eager work and
synchronisations between the replays, gives exactly the result of three eager calls.

Covered: loop_step in its resident and per-pass forms, loop_step_xi, loop_step_expanded,
ks_integrate, and the reverse-mode step's three calls (loop_cost_fwd, loop_cost_bwd,
loop_update_grad) in both layouts (the batched schedules are covered in test_gpu_batch.py)."""
import numpy as np
import pytest

import loopgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    from paper_2007_06427_amd import api as A
    torch.cuda.set_device(0)
    A.init()
    return A


def replay_equals_eager(call, state_eager, state_graph, reps=3):
    """call(state) queues one call on the current stream; states are tuples of tensors."""
    for _ in range(reps):
        call(state_eager)
    torch.cuda.synchronize()
    warm = tuple(t.clone() for t in state_graph)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call(warm)  # first call off the graph: one-time set-up happens here
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call(state_graph)
    for _ in range(reps):
        g.replay()
        torch.cuda.synchronize()
        _ = float(state_graph[0].abs().sum())  # unrelated eager work between the replays
    for a, b in zip(state_graph, state_eager):
        assert bool(torch.isfinite(a).all()), "the state left the stable range of the step"
        assert torch.equal(a, b)


def loops(Nx, Ns, n, seed, xi=False):
    rng = np.random.default_rng(seed)
    f = loopgen.random_xi_symmetric_field if xi else loopgen.random_band_field
    kx, ks = min(6, (Nx - 1) // 3), min(6, (Ns - 1) // 3)
    u = np.stack([f(rng, Nx, Ns, jmax=kx, kmax=ks, scale=0.3) for _ in range(n)])
    T = rng.uniform(30.0, 60.0, size=n)
    return torch.from_numpy(u).to(DEV), torch.from_numpy(T).to(DEV)


@pytest.mark.parametrize("Nx,Ns,n", [(32, 32, 2), (64, 128, 1)])
def test_loop_step(api, Nx, Ns, n):
    u, T = loops(Nx, Ns, n, seed=Nx)
    ws_e = api.Workspace(api.workspace_bytes(Nx, Ns, n))
    ws_g = api.Workspace(api.workspace_bytes(Nx, Ns, n))
    Je = torch.zeros(4, n, dtype=torch.float64, device=DEV)
    Jg = torch.zeros(4, n, dtype=torch.float64, device=DEV)
    replay_equals_eager(lambda st: api.loop_step(st[0], st[1], 22.0, 5e-5, api.IMEX, 4, J_hist=st[2],
                                                 ws=ws_e if st[2] is Je else ws_g),
                        (u.clone(), T.clone(), Je), (u.clone(), T.clone(), Jg))
    assert ws_g.status() == 0


def test_loop_step_xi(api):
    u, T = loops(64, 64, 3, seed=3, xi=True)
    ws = api.Workspace(api.xi_workspace_bytes(64, 64, 3))
    replay_equals_eager(lambda st: api.loop_step_xi(st[0], st[1], 39.0, 5e-4, api.IMEX, 3, ws=ws),
                        (u.clone(), T.clone()), (u.clone(), T.clone()))
    assert ws.status() == 0


def test_loop_step_expanded(api):
    u, T = loops(32, 64, 2, seed=4)
    ws = api.Workspace(api.workspace_bytes(32, 64, 2))
    replay_equals_eager(lambda st: api.loop_step_expanded(st[0], st[1], 22.0, 0.02, api.IMEX, 3, ws=ws),
                        (u.clone(), T.clone()), (u.clone(), T.clone()))
    assert ws.status() == 0


def test_ks_integrate(api):
    from paper_2007_06427_amd import initial_loops as il
    rng = np.random.default_rng(6)
    u0 = torch.from_numpy(np.stack([loopgen.random_ks_state(rng, 64, scale=0.5, odd=True) for _ in range(8)])).to(DEV)
    bufs = [(torch.zeros(8, 10, dtype=torch.float64, device=DEV),
             torch.zeros(8, 10, 33, dtype=torch.complex128, device=DEV)) for _ in range(2)]
    replay_equals_eager(lambda st: il.ks_integrate(st[0], 39.0, 0.05, 40, 4, True, st[1], st[2]),
                        (u0.clone(), *bufs[0]), (u0.clone(), *bufs[1]))


@pytest.mark.parametrize("layout", ["rfft", "band"])
def test_reverse_mode_step(api, layout):
    """One step of the autograd path as its three library calls: the forward (J, dJ/dT, the
    saved residual), the reverse pass (the gradient) and the update from the gradient."""
    Nx, Ns, L = 64, 256, 39.0
    u, T = loops(Nx, Ns, 2, seed=17)
    band = layout == "band"
    kw = {"layout": api.LAYOUT_BAND, "grid": (Nx, Ns)} if band else {}
    x = api.to_band(u) if band else u
    ws_e = api.Workspace(api.workspace_bytes(Nx, Ns, 2))
    ws_g = api.Workspace(api.workspace_bytes(Nx, Ns, 2))
    Je = torch.zeros(2, dtype=torch.float64, device=DEV)
    Jg = torch.zeros(2, dtype=torch.float64, device=DEV)

    def call(st):
        x, T, Jout = st
        ws = ws_e if Jout is Je else ws_g
        J, dJdT, rs = api.loop_cost_fwd(x, T, L, ws=ws, **kw)
        gu, gT = api.loop_cost_bwd(x, T, L, rs, dJdT, None, ws=ws, **kw)
        api.loop_update_grad(x, T, L, gu, gT, 5e-5, api.IMEX, **kw)
        Jout.copy_(J)

    replay_equals_eager(call, (x.clone(), T.clone(), Je), (x.clone(), T.clone(), Jg))
    assert ws_g.status() == 0
