"""GPU parity: each C-ABI entry point against the FP64 CPU oracle on the same seeded inputs.

Tolerance (set by the target accuracy of the method's hot path): 1e-12 relative, normwise,
in the norm of eq. inner_product_definition, per output and per step. For the scalar
dJ/dT = (1/T^2) <u_s, r>, which can be small next to its terms, the error is measured
against the Cauchy-Schwarz scale (L/T^2) ||u_s|| ||r||, the size of the terms that cancel.
"""
import json
import os

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


def wnorm(a, Nx):
    w = np.full(a.shape[-1], 2.0)
    w[0] = 1.0
    return np.sqrt(np.sum(w * np.abs(a) ** 2))


def relerr(a, b, Nx):
    return wnorm(a - b, Nx) / max(wnorm(b, Nx), 1e-300)


def make_batch(Nx, Ns, L, nloops, seed, kind="seeded"):
    """nloops loops of one shape. kind="seeded": low-mode spectrum; "full": whole band plus
    out-of-band garbage and a non-Hermitian column 0 (which the ABI must ignore)."""
    rng = np.random.default_rng(seed)
    us, Ts = [], []
    Kx, Ks = K.band_limits(Nx, Ns)
    for i in range(nloops):
        T = float(rng.uniform(20.0, 80.0))
        if kind == "seeded":
            u = loopgen.seeded_spectrum(rng, Nx, Ns, min(8, Kx), min(8, Ks), 0.5, 0.2)
        else:
            u = loopgen.random_band_field(rng, Nx, Ns, scale=0.3)
            junk = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
            u = u + 0.5 * junk * (~K.band_mask(Nx, Ns))
            u[:, 0] += 0.05 * (rng.standard_normal(Ns) + 1j * rng.standard_normal(Ns))
        us.append(u)
        Ts.append(T)
    return np.stack(us), np.array(Ts)


def to_dev(u, T):
    return (torch.from_numpy(np.ascontiguousarray(u)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(T)).to(DEV))


def dT_scale(u, T, L):
    uc = K.canonical(u)
    us = K.d_s(uc, L)
    r = K.residual(uc, T, L)
    return L / T ** 2 * np.sqrt(K.inner(us, us, L) / L * K.inner(r, r, L) / L)


SHAPES = [
    (32, 32, 22.0), (64, 128, 22.0), (64, 256, 39.0), (32, 64, 22.0), (64, 512, 39.0),
    (8, 8, 5.0), (16, 32, 9.0), (128, 64, 50.0), (1024, 16, 300.0), (8, 1024, 7.0), (512, 32, 150.0),
]


@pytest.mark.parametrize("Nx,Ns,L", SHAPES, ids=[f"{a}x{b}" for a, b, _ in SHAPES])
@pytest.mark.parametrize("kind", ["seeded", "full"])
def test_entry_points_match_oracle(api, Nx, Ns, L, kind):
    nl = 3
    u, T = make_batch(Nx, Ns, L, nl, seed=Nx * 7919 + Ns + (0 if kind == "seeded" else 1), kind=kind)
    ud, Td = to_dev(u, T)
    r = api.loop_residual(ud, Td, L).cpu().numpy()
    J = api.loop_cost(ud, Td, L).cpu().numpy()
    G, dJdT, J2 = (x.cpu().numpy() for x in api.loop_adjoint_grad(ud, Td, L))
    for i in range(nl):
        ro = K.residual(u[i], T[i], L)
        Go, dTo, Jo = K.adjoint_grad(u[i], T[i], L)
        assert relerr(r[i], ro, Nx) < TOL, ("r", i, relerr(r[i], ro, Nx))
        assert np.all(r[i][~K.band_mask(Nx, Ns)] == 0)
        assert abs(J[i] - Jo) <= TOL * Jo and abs(J2[i] - Jo) <= TOL * Jo
        assert relerr(G[i], Go, Nx) < TOL, ("G", i, relerr(G[i], Go, Nx))
        assert np.all(G[i][~K.band_mask(Nx, Ns)] == 0)
        assert abs(dJdT[i] - dTo) <= TOL * dT_scale(u[i], T[i], L), ("dJdT", i, dJdT[i], dTo)


@pytest.mark.parametrize("Nx,Ns,L", SHAPES[:6], ids=[f"{a}x{b}" for a, b, _ in SHAPES[:6]])
@pytest.mark.parametrize("scheme", [K.EXPLICIT, K.IMEX])
def test_one_step_matches_oracle(api, Nx, Ns, L, scheme):
    nl = 2
    u, T = make_batch(Nx, Ns, L, nl, seed=17 + Nx + Ns, kind="full")
    dtau = 1e-5 if scheme == K.EXPLICIT and Nx <= 32 else 5e-5
    if scheme == K.EXPLICIT:
        lm = K.lam(T.min(), L, Nx, Ns)
        dtau = min(dtau, 1.0 / np.max(np.abs(lm[K.band_mask(Nx, Ns)])))
    ud, Td = to_dev(u, T)
    Jh = torch.zeros(3, nl, dtype=torch.float64, device=DEV)
    api.loop_step(ud, Td, L, dtau, scheme, 3, J_hist=Jh)
    ug, Tg, Jg = ud.cpu().numpy(), Td.cpu().numpy(), Jh.cpu().numpy()
    for i in range(nl):
        uo, To, Jho = K.step(u[i], T[i], L, dtau, scheme, 3)
        assert relerr(ug[i], uo, Nx) < TOL, relerr(ug[i], uo, Nx)
        assert abs(Tg[i] - To) <= TOL * To
        assert np.all(np.abs(Jg[:, i] - Jho) <= TOL * Jho)
        assert np.all(ug[i][~K.band_mask(Nx, Ns)] == 0)


def test_full_size_large_batch_sampled(api):
    """256 x 1024, L = 100, 64 loops (the large batched workload): every loop is computed,
    and loops 0, 31 and 63 are checked against the oracle one by one."""
    specs = loopgen.config_loops(5)
    u = np.stack([s.uhat for s in specs])
    T = np.array([s.T for s in specs])
    L = specs[0].L
    ud, Td = to_dev(u, T)
    G, dJdT, J = (x.cpu().numpy() for x in api.loop_adjoint_grad(ud, Td, L))
    for i in (0, 31, 63):
        Go, dTo, Jo = K.adjoint_grad(u[i], T[i], L)
        assert relerr(G[i], Go, 256) < TOL
        assert abs(J[i] - Jo) <= TOL * Jo
        assert abs(dJdT[i] - dTo) <= TOL * dT_scale(u[i], T[i], L)
    assert np.all(np.isfinite(G)) and np.all(J > 0)


def test_full_size_translation_equivariance(api):
    """All 64 loops of 256 x 1024 (L = 100): the flow of a loop shifted in x by d and in s by
    sigma is the shifted flow, and J and dJ/dT do not change. A shift is a phase rotation
    exp(-i (q_j d + omega_k sigma)) of the spectrum, exact for band-limited fields, so any pass
    that mixed up an index, a sign or a conjugate half at full size would show here."""
    specs = loopgen.config_loops(5)
    u = np.stack([s.uhat for s in specs])
    T = np.array([s.T for s in specs])
    L = specs[0].L
    q, om = K.wavenumbers(L, 256, 1024)
    phase = np.exp(-1j * (q * (0.37 * L) + om * 0.19))
    ud, Td = to_dev(u, T)
    G, dJdT, J = (x.cpu().numpy() for x in api.loop_adjoint_grad(ud, Td, L))
    us, Ts = to_dev(u * phase, T)
    Gs, dJdTs, Js = (x.cpu().numpy() for x in api.loop_adjoint_grad(us, Ts, L))
    for i in range(len(specs)):
        assert relerr(Gs[i], G[i] * phase, 256) < TOL, (i, relerr(Gs[i], G[i] * phase, 256))
        assert abs(Js[i] - J[i]) <= TOL * J[i], i
        assert abs(dJdTs[i] - dJdT[i]) <= TOL * dT_scale(u[i], T[i], L), i


def test_batch_is_bitwise_equal_to_single_loops(api):
    Nx, Ns, L = 64, 128, 22.0
    u, T = make_batch(Nx, Ns, L, 5, seed=99)
    ud, Td = to_dev(u, T)
    G, dJdT, J = api.loop_adjoint_grad(ud, Td, L)
    for i in range(5):
        ui, Ti = to_dev(u[i:i + 1], T[i:i + 1])
        Gi, dJi, Ji = api.loop_adjoint_grad(ui, Ti, L)
        assert torch.equal(Gi[0], G[i]) and torch.equal(dJi[0], dJdT[i]) and torch.equal(Ji[0], J[i])


def test_deterministic(api):
    Nx, Ns, L = 64, 256, 39.0
    u, T = make_batch(Nx, Ns, L, 4, seed=5)
    outs = []
    for _ in range(2):
        ud, Td = to_dev(u, T)
        api.loop_step(ud, Td, L, 5e-5, K.IMEX, 4)
        outs.append((ud.clone(), Td.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_update_after_grad_equals_step(api):
    Nx, Ns, L = 32, 64, 22.0
    u, T = make_batch(Nx, Ns, L, 3, seed=3)
    for scheme in (K.EXPLICIT, K.IMEX):
        ud, Td = to_dev(u, T)
        ud2, Td2 = to_dev(u, T)
        G, dJdT, J = api.loop_adjoint_grad(ud, Td, L)
        api.loop_update(ud, Td, L, G, dJdT, 1e-5, scheme)
        api.loop_step(ud2, Td2, L, 1e-5, scheme, 1)
        a, b = ud.cpu().numpy(), ud2.cpu().numpy()
        for i in range(3):
            assert relerr(a[i], b[i], Nx) < 1e-14
        assert torch.allclose(Td, Td2, rtol=1e-15, atol=0)


def test_zero_steps_only_canonicalises(api):
    Nx, Ns, L = 32, 32, 22.0
    u, T = make_batch(Nx, Ns, L, 2, seed=8, kind="full")
    ud, Td = to_dev(u, T)
    api.loop_step(ud, Td, L, 1e-4, K.EXPLICIT, 0)
    got = ud.cpu().numpy()
    for i in range(2):
        assert np.abs(got[i] - K.canonical(u[i])).max() < 1e-16
    assert np.array_equal(Td.cpu().numpy(), T)


def test_nonpositive_period_sets_sticky_status(api):
    from paper_2007_06427_amd import _lib
    Nx, Ns, L = 32, 32, 22.0
    u, T = make_batch(Nx, Ns, L, 2, seed=1)
    ws = api.Workspace(api.workspace_bytes(Nx, Ns, 2))
    assert ws.status() == 0
    for bad in (-1.0, 0.0, float("nan")):
        ud, Td = to_dev(u, np.array([T[0], bad]))
        api.loop_cost(ud, Td, L, ws=ws)
        assert ws.status() == _lib.LOOP_ENONFINITE
        assert ws.status() == 0  # read clears it
    ud, Td = to_dev(u, T)
    api.loop_cost(ud, Td, L, ws=ws)
    assert ws.status() == 0


def test_explicit_blowup_is_flagged_not_silent(api):
    """Explicit Euler at dtau far beyond 2/|lambda|max diverges (the stiff q^8 term); the device
    flags the non-finite cost instead of returning garbage quietly."""
    from paper_2007_06427_amd import _lib
    spec = loopgen.config_loops(2)[0]
    ud, Td = to_dev(spec.uhat[None], np.array([spec.T]))
    ws = api.Workspace(api.workspace_bytes(spec.Nx, spec.Ns, 1))
    api.loop_step(ud, Td, spec.L, 1.0, K.EXPLICIT, 40, ws=ws)
    assert ws.status() == _lib.LOOP_ENONFINITE


HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_trajectory_plain32x32_2000_explicit_steps(api):
    """The 32 x 32 workload: 2000 explicit steps at dtau = 1e-4 against the stored oracle run."""
    g = json.load(open(os.path.join(HERE, "oracle_traj_plain32x32.json")))
    spec = loopgen.config_loops(1)[0]
    ud, Td = to_dev(spec.uhat[None], np.array([spec.T]))
    Jh = torch.zeros(g["steps"], 1, dtype=torch.float64, device=DEV)
    api.loop_step(ud, Td, spec.L, g["dtau"], K.EXPLICIT, g["steps"], J_hist=Jh)
    Jh = Jh.cpu().numpy()[:, 0]
    for m, v in g["J_hist_marks"].items():
        assert abs(Jh[int(m)] - v) <= 1e-10 * v
    assert abs(Td.item() - g["T_final"]) <= 1e-10 * g["T_final"]
    uo = np.zeros_like(spec.uhat)
    for j, k, re, im in g["uhat_final_band"]:
        uo[k % spec.Ns, j] = complex(re, im)
    assert relerr(ud.cpu().numpy()[0], uo, spec.Nx) < 1e-10
    assert np.all(np.diff(Jh) <= 0)


def test_trajectory_plain64x128_imex(api):
    g = json.load(open(os.path.join(HERE, "oracle_traj_plain64x128_200.json")))
    spec = loopgen.config_loops(2)[0]
    ud, Td = to_dev(spec.uhat[None], np.array([spec.T]))
    Jh = torch.zeros(g["steps"], 1, dtype=torch.float64, device=DEV)
    api.loop_step(ud, Td, spec.L, g["dtau"], K.IMEX, g["steps"], J_hist=Jh)
    Jh = Jh.cpu().numpy()[:, 0]
    for m, v in g["J_hist_marks"].items():
        assert abs(Jh[int(m)] - v) <= 1e-10 * v
    assert abs(Td.item() - g["T_final"]) <= 1e-10 * g["T_final"]
    assert np.all(np.diff(Jh) <= 0)


def test_log_plain64x128_20000_imex_steps(api):
    """The 64 x 128 workload as specified: 20 000 IMEX steps at dtau = 5e-5 from its seed, J(tau)
    and T(tau) every 10 steps against the oracle's stored log, to 1e-10, and the end state."""
    g = json.load(open(os.path.join(HERE, "oracle_traj_plain64x128.json")))
    spec = loopgen.config_loops(2)[0]
    ud, Td = to_dev(spec.uhat[None], np.array([spec.T]))
    every, n = g["log_every"], len(g["J_log"])
    Jh = torch.zeros(g["steps"], 1, dtype=torch.float64, device=DEV)
    Tl = torch.zeros(n, dtype=torch.float64, device=DEV)
    ws = api.Workspace(api.workspace_bytes(spec.Nx, spec.Ns, 1))
    for i in range(n):
        Tl[i].copy_(Td[0])
        api.loop_step(ud, Td, spec.L, g["dtau"], K.IMEX, every, J_hist=Jh[i * every:(i + 1) * every], ws=ws)
    assert ws.status() == 0
    J = Jh.cpu().numpy()[::every, 0]
    Jo, To = np.array(g["J_log"]), np.array(g["T_log"])
    assert np.max(np.abs(J - Jo) / Jo) <= 1e-10, np.max(np.abs(J - Jo) / Jo)
    assert np.max(np.abs(Tl.cpu().numpy() - To) / To) <= 1e-10
    assert abs(Td.item() - g["T_final"]) <= 1e-10 * g["T_final"]
    assert abs(api.loop_cost(ud, Td, spec.L).item() - g["J_final"]) <= 1e-10 * g["J_final"]
    uo = np.zeros_like(spec.uhat)
    for j, k, re, im in g["uhat_final_band"]:
        uo[k % spec.Ns, j] = complex(re, im)
    assert relerr(ud.cpu().numpy()[0], uo, spec.Nx) < 1e-10
    assert np.all(np.diff(Jh.cpu().numpy()[:, 0]) <= 0)


@pytest.mark.parametrize("form", [0, 2])
def test_reaches_the_oracle_converged_state(api, form):
    """Convergence parity: from the 32 x 32 workload's seed, IMEX at dtau = 0.05, the oracle
    needed the stored number of steps to bring J below 1e-10 (it ends on an equilibrium).
    The GPU run of the same steps must end with J < 1e-10, T within 1e-8 of the oracle's,
    and the same band-mode magnitudes (invariant under the x- and s-shifts that leave J
    unchanged) to 1e-8."""
    g = json.load(open(os.path.join(HERE, "oracle_converged_plain32x32.json")))
    spec = loopgen.config_loops(1)[0]
    assert (spec.Nx, spec.Ns, spec.L, spec.T) == (g["Nx"], g["Ns"], g["L"], g["T0"])
    ud, Td = to_dev(spec.uhat[None], np.array([spec.T]))
    prev = api.set_resident(form)  # 0: per-pass kernels, 2: the LDS-resident kernel
    try:
        assert api.step_form(spec.Nx, spec.Ns) == ("resident" if form == 2 else "per-pass")
        api.loop_step(ud, Td, spec.L, g["dtau"], K.IMEX, g["steps"])
    finally:
        api.set_resident(prev)
    J = api.loop_cost(ud, Td, spec.L).item()
    assert J < g["J_tol"], J
    assert abs(J - g["J_final"]) <= 1e-3 * g["J_final"]
    assert abs(Td.item() - g["T_final"]) <= 1e-8
    u = ud.cpu().numpy()[0]
    worst = max(abs(abs(u[k % spec.Ns, j]) - a) for j, k, a in g["abs_uhat_final_band"])
    assert worst <= 1e-8, worst
    assert g["end_state"] == "equilibrium"
