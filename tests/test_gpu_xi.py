"""GPU tests of the centre-symmetric form loop_step_xi (Sec. 3, eq. KS_loop_sym; half the
state and traffic for loops with u odd in x).

On centre-symmetric inputs it must match the oracle's step to 1e-12 per step (normwise, as in
test_gpu_parity.py), and loop_step to rounding. On other inputs it steps their orthogonal
projection onto centre-symmetric loops (oracle xi_project), and its outputs are
centre-symmetric exactly.
"""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SHAPES = [(8, 8), (16, 32), (32, 64), (64, 128), (32, 1024), (128, 64), (512, 16), (64, 512), (256, 256)]


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


def xi(u):
    k_neg = (-np.arange(u.shape[0])) % u.shape[0]
    return -np.conj(u[k_neg, :])


def loops(Nx, Ns, n, seed, scale=0.3, jmax=None, kmax=None):
    rng = np.random.default_rng(seed)
    u = np.stack([loopgen.random_xi_symmetric_field(rng, Nx, Ns, jmax=jmax, kmax=kmax, scale=scale)
                  for _ in range(n)])
    return u, rng.uniform(20.0, 80.0, size=n)


def run_xi(api, u, T, L, dtau, scheme, nsteps):
    ud = torch.from_numpy(u).to(DEV)
    Td = torch.tensor(T, dtype=torch.float64, device=DEV)
    Jh = torch.zeros(max(nsteps, 1), len(T), dtype=torch.float64, device=DEV)
    Nx = 2 * (u.shape[2] - 1)
    ws = api.Workspace(api.xi_workspace_bytes(Nx, u.shape[1], len(T)))
    api.loop_step_xi(ud, Td, L, dtau, scheme, nsteps, J_hist=Jh, ws=ws)
    torch.cuda.synchronize()
    assert ws.status() == 0
    return ud.cpu().numpy(), Td.cpu().numpy(), Jh.cpu().numpy()


@pytest.mark.parametrize("Nx,Ns", SHAPES)
@pytest.mark.parametrize("scheme", [0, 1])
def test_one_step_matches_oracle(api, Nx, Ns, scheme):
    u, T = loops(Nx, Ns, 2, seed=Nx * 7 + Ns)
    L = 22.0 if Nx <= 64 else 60.0
    dtau = 5e-5 if scheme == 1 else 1e-8
    ug, Tg, Jg = run_xi(api, u, T, L, dtau, scheme, 1)
    for i in range(2):
        uo, To, Jo = K.step(u[i], T[i], L, dtau, scheme, 1)
        assert wrel(ug[i], uo) < 1e-12, (Nx, Ns)
        assert abs(Tg[i] - To) <= 1e-12 * abs(To)
        assert abs(Jg[0, i] - Jo[0]) <= 1e-12 * Jo[0]
        assert np.array_equal(xi(ug[i]), ug[i])  # centre-symmetric exactly


@pytest.mark.parametrize("Nx,Ns", [(32, 64), (64, 128), (256, 256)])
def test_five_steps_match_oracle_and_full_path(api, Nx, Ns):
    # low modes only, so that the loops stay smooth enough for T to stay positive
    u, T = loops(Nx, Ns, 2, seed=3 + Nx, jmax=min(10, (Nx - 1) // 3), kmax=min(10, (Ns - 1) // 3))
    L = 39.0
    ug, Tg, Jg = run_xi(api, u, T, L, 5e-5, 1, 5)
    uf = torch.from_numpy(u).to(DEV)
    Tf = torch.tensor(T, dtype=torch.float64, device=DEV)
    Jf = torch.zeros(5, 2, dtype=torch.float64, device=DEV)
    api.loop_step(uf, Tf, L, 5e-5, 1, 5, J_hist=Jf)
    uf, Tf, Jf = uf.cpu().numpy(), Tf.cpu().numpy(), Jf.cpu().numpy()
    for i in range(2):
        uo, To, Jo = K.step(u[i], T[i], L, 5e-5, K.IMEX, 5)
        assert wrel(ug[i], uo) < 1e-11
        assert abs(Tg[i] - To) <= 1e-11 * abs(To)
        assert np.allclose(Jg[:, i], Jo, rtol=1e-11, atol=0)
        assert wrel(ug[i], uf[i]) < 1e-13
        assert np.allclose(Jg[:, i], Jf[:, i], rtol=1e-13, atol=0)


def test_projects_other_inputs(api):
    rng = np.random.default_rng(9)
    Nx, Ns, L = 32, 64, 22.0
    u = np.stack([loopgen.random_band_field(rng, Nx, Ns, scale=0.3) for _ in range(2)])
    T = np.array([30.0, 45.0])
    u0, T0, _ = run_xi(api, u, T, L, 5e-5, 1, 0)
    for i in range(2):
        assert np.abs(u0[i] - K.xi_project(u[i])).max() <= 1e-16 * np.abs(u[i]).max()
    assert np.array_equal(T0, T)
    u1, T1, J1 = run_xi(api, u, T, L, 5e-5, 1, 2)
    for i in range(2):
        uo, To, Jo = K.step(K.xi_project(u[i]), T[i], L, 5e-5, K.IMEX, 2)
        assert wrel(u1[i], uo) < 1e-12
        assert abs(T1[i] - To) <= 1e-12 * To


def test_many_loops_agree_with_single_runs(api):
    u, T = loops(64, 64, 5, seed=21)
    ub, Tb, Jb = run_xi(api, u, T, 39.0, 5e-5, 1, 3)
    for i in range(5):
        ui, Ti, Ji = run_xi(api, u[i:i + 1], T[i:i + 1], 39.0, 5e-5, 1, 3)
        assert wrel(ub[i], ui[0]) < 1e-14
        assert abs(Tb[i] - Ti[0]) <= 1e-14 * Ti[0]
        assert np.allclose(Jb[:, i], Ji[:, 0], rtol=1e-14, atol=0)


def test_workspace_is_about_half(api):
    for (Nx, Ns, n) in [(64, 64, 256), (256, 1024, 64), (32, 512, 10)]:
        assert api.xi_workspace_bytes(Nx, Ns, n) <= 0.6 * api.workspace_bytes(Nx, Ns, n)


def test_rejects_rows_longer_than_512(api):
    rng = np.random.default_rng(1)
    u = loopgen.random_xi_symmetric_field(rng, 1024, 8)[None]
    with pytest.raises(api.LoopOrbitError):
        run_xi(api, u, np.array([30.0]), 22.0, 5e-5, 1, 1)
