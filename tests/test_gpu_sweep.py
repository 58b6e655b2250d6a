"""GPU parity over a seeded sweep of shapes: 24 draws of (Nx, Ns) from the powers of two 8..1024
with Nx Ns <= 65536, L proportional to Nx (0.15 Nx to 0.6 Nx, the resolution of the paper's
loops), T in [15, 150], and fields either low-mode or filling the whole band (with out-of-band
entries and a non-Hermitian column 0 that the ABI ignores).

Per loop, against the FP64 oracle: loop_adjoint_grad (G, J, dJ/dT) and one IMEX loop_step to
1e-12 relative (normwise; dJ/dT against the size of the terms that cancel in it, as in
test_gpu_parity.py); and the loops with Nx <= 512 as one ragged batch, one step each, to
1e-12 against the oracle's step."""
import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
DEV = "cuda:0"
POW = [8, 16, 32, 64, 128, 256, 512, 1024]


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


def sweep(n=24, seed=2007):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        Nx, Ns = int(rng.choice(POW)), int(rng.choice(POW))
        if Nx * Ns > 65536:
            continue
        L = float(Nx * rng.uniform(0.15, 0.6))
        T = float(rng.uniform(15.0, 150.0))
        if len(out) % 2 == 0:
            Kx, Ks = K.band_limits(Nx, Ns)
            u = loopgen.seeded_spectrum(rng, Nx, Ns, min(8, Kx), min(8, Ks), 0.5, 0.2)
        else:
            u = loopgen.random_band_field(rng, Nx, Ns, scale=0.3)
            u = u + 0.5 * (rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)) * (~K.band_mask(Nx, Ns))
            u[:, 0] += 0.05 * (rng.standard_normal(Ns) + 1j * rng.standard_normal(Ns))
        out.append((Nx, Ns, L, T, u))
    return out


SWEEP = sweep()


@pytest.mark.parametrize("i", range(len(SWEEP)), ids=[f"{s[0]}x{s[1]}" for s in SWEEP])
def test_grad_and_step_match_oracle(api, i):
    Nx, Ns, L, T, u = SWEEP[i]
    ud = torch.from_numpy(u[None].copy()).to(DEV)
    Td = torch.tensor([T], dtype=torch.float64, device=DEV)
    G, dJdT, J = (x.cpu().numpy() for x in api.loop_adjoint_grad(ud, Td, L))
    Go, dTo, Jo = K.adjoint_grad(u, T, L)
    assert wrel(G[0], Go) < TOL, wrel(G[0], Go)
    assert np.all(G[0][~K.band_mask(Nx, Ns)] == 0)
    assert abs(J[0] - Jo) <= TOL * Jo
    assert abs(dJdT[0] - dTo) <= TOL * dT_scale(u, T, L)
    dtau = 1e-4
    api.loop_step(ud, Td, L, dtau, api.IMEX, 1)
    uo, To, _ = K.step(u, T, L, dtau, api.IMEX, 1)
    assert wrel(ud.cpu().numpy()[0], uo) < TOL
    assert abs(Td.item() - To) <= TOL * To


def test_sweep_as_one_ragged_batch(api):
    loops = [s for s in SWEEP if s[0] <= 512]
    assert len(loops) >= 16
    b = api.Batch([(L, Nx, Ns) for (Nx, Ns, L, T, u) in loops])
    pool = b.pack([torch.from_numpy(u) for (*_, u) in loops])
    T = torch.tensor([s[3] for s in loops], dtype=torch.float64, device=DEV)
    dtau = 1e-4
    b.step(pool, T, dtau, api.IMEX, 1)
    torch.cuda.synchronize()
    assert b.status() == 0
    for (Nx, Ns, L, T0, u), got, Tg in zip(loops, b.unpack(pool), T.cpu().numpy()):
        uo, To, _ = K.step(u, T0, L, dtau, api.IMEX, 1)
        assert wrel(got.cpu().numpy(), uo) < TOL, (Nx, Ns, wrel(got.cpu().numpy(), uo))
        assert abs(Tg - To) <= TOL * To
