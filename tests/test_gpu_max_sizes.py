"""Parity at the largest sizes each entry point takes, against the oracle (a few loops each, so
the oracle finishes in seconds):

* loop_residual, loop_cost, loop_adjoint_grad and loop_step at Nx = Ns = 1024, the largest
  shape of the uniform entry points, and the reverse mode (loop_cost_fwd / loop_cost_bwd, with
  and without the kept u, both layouts) there and at the smallest shape, 8 x 8;
* a ragged batch holding the largest (512 x 1024) and the smallest (8 x 8) shapes a plan
  takes, with the two mixed extremes 8 x 1024 and 512 x 8;
* loop_step_xi and loop_expanded_grad at 512 x 1024, their largest shape;
* the largest loop count, 65535 loops of 8 x 8, per loop and as a batched plan.

The tolerance is that of the other parity tests: 1e-12 normwise per output and per step. dJ/dT
is measured against the size of the terms that cancel in it, (L/T^2) ||u_s|| ||r||."""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
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


def dT_scale(u, T, L):
    uc = K.canonical(u)
    us, r = K.d_s(uc, L), K.residual(uc, T, L)
    return L / T ** 2 * np.sqrt(K.inner(us, us, L) / L * K.inner(r, r, L) / L)


def loops_1024(seed):
    """A low-mode loop and a whole-band loop with out-of-band entries (which the ABI ignores)."""
    rng = np.random.default_rng(seed)
    Nx = Ns = 1024
    u0 = loopgen.seeded_spectrum(rng, Nx, Ns, 8, 8, 0.5, 0.2)
    u1 = loopgen.random_band_field(rng, Nx, Ns, scale=0.2)
    u1 = u1 + 0.5 * (rng.standard_normal(u1.shape) + 1j * rng.standard_normal(u1.shape)) * (~K.band_mask(Nx, Ns))
    return np.stack([u0, u1]), np.array([37.0, 71.0])


def test_uniform_entry_points_at_1024x1024(api):
    u, T = loops_1024(1024)
    L = 300.0
    print(f"1024 x 1024, L = {L}, 2 loops", flush=True)
    ud, Td = torch.from_numpy(u).to(DEV), torch.from_numpy(T).to(DEV)
    r = api.loop_residual(ud, Td, L).cpu().numpy()
    J = api.loop_cost(ud, Td, L).cpu().numpy()
    G, dJdT, J2 = (x.cpu().numpy() for x in api.loop_adjoint_grad(ud, Td, L))
    for i in range(2):
        ro = K.residual(u[i], T[i], L)
        Go, dTo, Jo = K.adjoint_grad(u[i], T[i], L)
        assert wrel(r[i], ro) < TOL, ("r", i, wrel(r[i], ro))
        assert np.all(r[i][~K.band_mask(1024, 1024)] == 0)
        assert abs(J[i] - Jo) <= TOL * Jo and abs(J2[i] - Jo) <= TOL * Jo
        assert wrel(G[i], Go) < TOL, ("G", i, wrel(G[i], Go))
        assert np.all(G[i][~K.band_mask(1024, 1024)] == 0)
        assert abs(dJdT[i] - dTo) <= TOL * dT_scale(u[i], T[i], L)


def test_step_at_1024x1024(api):
    u, T = loops_1024(2048)
    L, dtau = 300.0, 5e-5
    ud, Td = torch.from_numpy(u).to(DEV), torch.from_numpy(T).to(DEV)
    Jh = torch.zeros(1, 2, dtype=torch.float64, device=DEV)
    api.loop_step(ud, Td, L, dtau, api.IMEX, 1, J_hist=Jh)
    ug, Tg, Jg = ud.cpu().numpy(), Td.cpu().numpy(), Jh.cpu().numpy()
    for i in range(2):
        uo, To, Jo = K.step(u[i], T[i], L, dtau, K.IMEX, 1)
        assert wrel(ug[i], uo) < TOL, (i, wrel(ug[i], uo))
        assert abs(Tg[i] - To) <= TOL * To
        assert abs(Jg[0, i] - Jo[0]) <= TOL * Jo[0]


def test_ragged_batch_at_its_extremes(api):
    rng = np.random.default_rng(4096)
    shapes = [(150.0, 512, 1024), (9.0, 8, 8), (7.0, 8, 1024), (150.0, 512, 8)]
    us = [loopgen.seeded_spectrum(rng, Nx, Ns, min(8, K.band_limits(Nx, Ns)[0]), min(8, K.band_limits(Nx, Ns)[1]),
                                  0.5, 0.2) for (_, Nx, Ns) in shapes]
    Ts = rng.uniform(20.0, 80.0, size=len(shapes))
    b = api.Batch(shapes)
    pool = b.pack([torch.from_numpy(u) for u in us])
    T = torch.from_numpy(Ts.copy()).to(DEV)
    Jh = torch.zeros(2, len(shapes), dtype=torch.float64, device=DEV)
    b.step(pool, T, 5e-5, api.IMEX, 2, J_hist=Jh)
    torch.cuda.synchronize()
    assert b.status() == 0
    ub, Tb, Jb = [x.cpu().numpy() for x in b.unpack(pool)], T.cpu().numpy(), Jh.cpu().numpy()
    for i, (L, Nx, Ns) in enumerate(shapes):
        uo, To, Jo = K.step(us[i], Ts[i], L, 5e-5, K.IMEX, 2)
        assert wrel(ub[i], uo) < TOL, (Nx, Ns, wrel(ub[i], uo))
        assert abs(Tb[i] - To) <= TOL * To
        assert np.all(np.abs(Jb[:, i] - Jo) <= TOL * Jo)


def test_xi_step_at_512x1024(api):
    rng = np.random.default_rng(512)
    Nx, Ns, L = 512, 1024, 60.0
    u = np.stack([loopgen.random_xi_symmetric_field(rng, Nx, Ns, jmax=10, kmax=10, scale=0.3) for _ in range(2)])
    T = rng.uniform(20.0, 80.0, size=2)
    ud, Td = torch.from_numpy(u).to(DEV), torch.from_numpy(T.copy()).to(DEV)
    Jh = torch.zeros(1, 2, dtype=torch.float64, device=DEV)
    ws = api.Workspace(api.xi_workspace_bytes(Nx, Ns, 2))
    api.loop_step_xi(ud, Td, L, 5e-5, api.IMEX, 1, J_hist=Jh, ws=ws)
    torch.cuda.synchronize()
    assert ws.status() == 0
    ug, Tg, Jg = ud.cpu().numpy(), Td.cpu().numpy(), Jh.cpu().numpy()
    for i in range(2):
        uo, To, Jo = K.step(u[i], T[i], L, 5e-5, K.IMEX, 1)
        assert wrel(ug[i], uo) < TOL
        assert abs(Tg[i] - To) <= TOL * To
        assert abs(Jg[0, i] - Jo[0]) <= TOL * Jo[0]


def test_expanded_grad_at_512x1024(api):
    rng = np.random.default_rng(1536)
    Nx, Ns, L = 512, 1024, 60.0
    u = np.stack([loopgen.random_band_field(rng, Nx, Ns, scale=0.4) for _ in range(2)])
    T = np.array([33.0, 58.0])
    G, dT, J = (x.cpu().numpy() for x in api.loop_expanded_grad(torch.from_numpy(u).to(DEV),
                                                                 torch.from_numpy(T).to(DEV), L))
    for i in range(2):
        Go, dTo, Jo = K.expanded_grad(u[i], T[i], L)
        assert wrel(G[i], Go) < TOL
        assert abs(dT[i] - dTo) <= TOL * dT_scale(u[i], T[i], L)
        assert abs(J[i] - Jo) <= TOL * Jo


@pytest.mark.parametrize("Nx,Ns", [(1024, 1024), (8, 8), (16, 1024)])
def test_reverse_mode_at_the_extremes(api, Nx, Ns):
    """The reverse pass in both layouts, with and without the forward's u on the s grid,
    gives -gJ w_j L G_1 of loop_adjoint_grad bit for bit and the oracle's gradient to 1e-12."""
    rng = np.random.default_rng(Nx + Ns)
    L = 300.0 if Nx == 1024 else 22.0
    u = np.stack([loopgen.random_band_field(rng, Nx, Ns, scale=0.2) for _ in range(2)])
    T = np.array([37.0, 71.0])
    print(f"{Nx} x {Ns}, L = {L}, 2 loops", flush=True)
    ud, Td = torch.from_numpy(u).to(DEV), torch.from_numpy(T).to(DEV)
    gJ = torch.tensor([1.0, -0.5], dtype=torch.float64, device=DEV)
    G, dJdT, J = api.loop_adjoint_grad(ud, Td, L)
    w = torch.full((u.shape[-1],), 2.0, dtype=torch.float64, device=DEV)
    w[0] = 1.0
    want = -(gJ[:, None, None] * L) * w * G
    for layout in ("rfft", "band"):
        kw = {"layout": api.LAYOUT_BAND, "grid": (Nx, Ns)} if layout == "band" else {}
        x = api.to_band(ud) if layout == "band" else ud
        for keep in (False, True):
            us = api.saved_u(2, Nx, Ns, DEV) if keep else None
            J2, dJdT2, rs = api.loop_cost_fwd(x, Td, L, usave=us, **kw)
            gu, gT = api.loop_cost_bwd(x, Td, L, rs, dJdT2, gJ, usave=us, **kw)
            assert torch.equal(J2, J) and torch.equal(dJdT2, dJdT), (layout, keep)
            g = api.from_band(gu, Nx, Ns) if layout == "band" else gu
            assert torch.equal(g, want), (layout, keep)
            assert torch.equal(gT, gJ * dJdT)
    Gn = G.cpu().numpy()
    for i in range(2):
        Go, dTo, Jo = K.adjoint_grad(u[i], T[i], L)
        assert wrel(Gn[i], Go) < TOL


def test_largest_loop_count(api):
    """65535 loops (the most one call or plan takes) of 8 x 8: one IMEX step of every loop by
    loop_step, and the same loops as a batched plan (a loop's index then fills the 16 bits the
    batched item codes give it). Sampled loops (the first, the last and others) of both against
    the oracle's step to 1e-12; the batch against loop_step to 1e-12 on every loop (loop_step
    packs rows of neighbouring loops into one transform, the batch rows of one loop, so they
    agree to rounding); the persistent schedule equal to the per-pass one bit for bit."""
    n, Nx, Ns, L, dtau = 65535, 8, 8, 5.0, 1e-3
    rng = np.random.default_rng(65535)
    band = K.band_mask(Nx, Ns)
    u = (rng.standard_normal((n, Ns, Nx // 2 + 1)) + 1j * rng.standard_normal((n, Ns, Nx // 2 + 1))) * 0.3 * band
    T = rng.uniform(10.0, 30.0, n)
    ud = torch.from_numpy(u).to(DEV)
    Td = torch.from_numpy(T).to(DEV)
    api.loop_step(ud, Td, L, dtau, api.IMEX, 1)
    torch.cuda.synchronize()
    uo, To = ud.cpu().numpy(), Td.cpu().numpy()
    b = api.Batch([(L, Nx, Ns)] * n)
    assert b.offsets[-1] == (n - 1) * Ns * (Nx // 2 + 1)  # one shape: the pool is the loops back to back
    out = {}
    for schedule in (api.Batch.PER_PASS, api.Batch.PERSISTENT):
        b.set_schedule(schedule)
        pool = torch.from_numpy(u.reshape(-1).copy()).to(DEV)
        Tb = torch.from_numpy(T.copy()).to(DEV)
        b.step(pool, Tb, dtau, api.IMEX, 1)
        torch.cuda.synchronize()
        assert b.status() == 0
        out[schedule] = (pool.cpu().numpy().reshape(u.shape), Tb.cpu().numpy())
    ub, Tbatch = out[api.Batch.PER_PASS]
    assert np.array_equal(out[api.Batch.PERSISTENT][0], ub) and np.array_equal(out[api.Batch.PERSISTENT][1], Tbatch)
    w = np.full(Nx // 2 + 1, 2.0)
    w[0] = 1.0
    diff = np.sqrt(np.sum(w * np.abs(ub - uo) ** 2, axis=(1, 2)) / np.sum(w * np.abs(uo) ** 2, axis=(1, 2)))
    assert diff.max() < TOL, (int(diff.argmax()), diff.max())
    assert np.all(np.abs(Tbatch - To) <= TOL * To)
    for i in [0, 1, 2, 255, 256, 32767, n - 3, n - 2, n - 1] + list(rng.integers(0, n, 16)):
        ue, Te, _ = K.step(u[i], T[i], L, dtau, api.IMEX, 1)
        for got, Tg in ((uo[i], To[i]), (ub[i], Tbatch[i])):
            assert wrel(got, ue) < TOL, (i, wrel(got, ue))
            assert abs(Tg - Te) <= TOL * Te, i
