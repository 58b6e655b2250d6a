"""Tensor-level binding of the C ABI. Every function takes device tensors and queues work
on the current torch stream.

Shapes: uhat is complex128 of shape (nloops, Ns, Nx//2 + 1) or (Ns, Nx//2 + 1), in the rfft
layout of include/looporbit.h. T is float64 of shape (nloops,). Torch provides device memory
and streams only. All arithmetic runs in liblooporbit.so.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Tuple

import torch

from . import _lib
from ._lib import EXPLICIT, IMEX, LAYOUT_BAND, LAYOUT_RFFT, LoopOrbitError, check  # noqa: F401

_WS: Dict[Tuple[int, int], "Workspace"] = {}


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def shape_of(uhat: torch.Tensor):
    """(nloops, Nx, Ns) of an rfft-layout tensor, which must be a contiguous complex128 CUDA tensor."""
    if uhat.dtype != torch.complex128:
        raise TypeError("uhat must be complex128")
    if not uhat.is_cuda:
        raise ValueError("uhat must be a device tensor")
    if not uhat.is_contiguous():
        raise ValueError("uhat must be contiguous")
    if uhat.dim() == 2:
        nl, Ns, H = 1, uhat.shape[0], uhat.shape[1]
    elif uhat.dim() == 3:
        nl, Ns, H = uhat.shape
    else:
        raise ValueError("uhat must be (Ns, Nx//2+1) or (nloops, Ns, Nx//2+1)")
    return int(nl), 2 * (int(H) - 1), int(Ns)


def _periods(T, nl, device):
    if not isinstance(T, torch.Tensor):
        T = torch.full((nl,), float(T), dtype=torch.float64, device=device)
    if T.dtype != torch.float64 or not T.is_cuda or not T.is_contiguous() or T.numel() != nl:
        raise ValueError("T must be a contiguous float64 device tensor with one entry per loop")
    return T


def workspace_bytes(Nx: int, Ns: int, nloops: int) -> int:
    n = ctypes.c_size_t(0)
    check(_lib.lib().loop_workspace_bytes(Nx, Ns, nloops, ctypes.byref(n)), "loop_workspace_bytes")
    return int(n.value)


class Workspace:
    """A device work space (caller-owned memory of the C ABI), prepared by loop_workspace_init."""

    def __init__(self, nbytes: int, device=None):
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.nbytes = int(self.buf.numel())
        check(_lib.lib().loop_workspace_init(_ptr(self.buf), self.nbytes, _stream_ptr()), "loop_workspace_init")

    @property
    def ptr(self):
        return _ptr(self.buf)

    def status(self) -> int:
        """Read and clear the sticky device status (synchronises the current stream)."""
        return int(_lib.lib().loop_status_sync(self.ptr, _stream_ptr()))


def workspace(Nx: int, Ns: int, nloops: int, device=None) -> Workspace:
    """A cached work space big enough for (Nx, Ns, nloops) on the current device."""
    need = workspace_bytes(Nx, Ns, nloops)
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    key = (dev, 0)
    ws = _WS.get(key)
    if ws is None or ws.nbytes < need:
        ws = Workspace(need, device=torch.device("cuda", dev))
        _WS[key] = ws
    return ws


def init() -> None:
    check(_lib.lib().loop_init(), "loop_init")


def loop_residual(uhat: torch.Tensor, T, L: float, out: torch.Tensor = None, ws: Workspace = None) -> torch.Tensor:
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    out = torch.empty_like(uhat) if out is None else out
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_residual(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(out), ws.ptr, ws.nbytes,
                                   _stream_ptr()), "loop_residual")
    return out


def loop_cost(uhat: torch.Tensor, T, L: float, out: torch.Tensor = None, ws: Workspace = None) -> torch.Tensor:
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    out = torch.empty(nl, dtype=torch.float64, device=uhat.device) if out is None else out
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_cost(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(out), ws.ptr, ws.nbytes,
                               _stream_ptr()), "loop_cost")
    return out


def loop_adjoint_grad(uhat: torch.Tensor, T, L: float, ws: Workspace = None):
    """Returns (G1_hat, dJ/dT, J): the flow's field component, the period derivative and the cost."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    G = torch.empty_like(uhat)
    dJdT = torch.empty(nl, dtype=torch.float64, device=uhat.device)
    J = torch.empty(nl, dtype=torch.float64, device=uhat.device)
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_adjoint_grad(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(G), _ptr(dJdT), _ptr(J),
                                       ws.ptr, ws.nbytes, _stream_ptr()), "loop_adjoint_grad")
    return G, dJdT, J


def loop_cost_grad(uhat: torch.Tensor, T, L: float, gJ: torch.Tensor = None, ws: Workspace = None):
    """(grad_uhat, grad_T) of sum_l gJ[l] J_l in torch's complex convention (see the C header)."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    if gJ is not None and (gJ.dtype != torch.float64 or gJ.numel() != nl or not gJ.is_contiguous()):
        raise ValueError("gJ must be a contiguous float64 tensor with one entry per loop")
    gu = torch.empty_like(uhat)
    gT = torch.empty(nl, dtype=torch.float64, device=uhat.device)
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_cost_grad(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(gJ) if gJ is not None else None,
                                    _ptr(gu), _ptr(gT), ws.ptr, ws.nbytes, _stream_ptr()), "loop_cost_grad")
    return gu, gT


def band_dims(Nx: int, Ns: int):
    """(C, NB): retained spatial modes j = 0..Kx and temporal modes |k| <= Ks of the band layout."""
    return (Nx - 1) // 3 + 1, 2 * ((Ns - 1) // 3) + 1


def band_shape_of(ub: torch.Tensor, Nx: int, Ns: int) -> int:
    """nloops of a band-layout tensor (nloops, C, NB) or (C, NB) for an Nx x Ns grid."""
    C, NB = band_dims(Nx, Ns)
    if ub.dtype != torch.complex128 or not ub.is_cuda or not ub.is_contiguous():
        raise ValueError("band-layout state must be a contiguous complex128 device tensor")
    if tuple(ub.shape[-2:]) != (C, NB) or ub.dim() not in (2, 3):
        raise ValueError(f"band-layout state must be (nloops, {C}, {NB}) or ({C}, {NB}) for {Nx} x {Ns}")
    return 1 if ub.dim() == 2 else int(ub.shape[0])


def to_band(uhat: torch.Tensor) -> torch.Tensor:
    """rfft layout -> band layout (nloops, C, NB), column 0 made Hermitian."""
    nl, Nx, Ns = shape_of(uhat)
    C, NB = band_dims(Nx, Ns)
    ub = torch.empty((nl, C, NB) if uhat.dim() == 3 else (C, NB), dtype=torch.complex128, device=uhat.device)
    check(_lib.lib().loop_to_band(Nx, Ns, nl, _ptr(uhat), _ptr(ub), _stream_ptr()), "loop_to_band")
    return ub


def from_band(ub: torch.Tensor, Nx: int, Ns: int) -> torch.Tensor:
    """band layout -> rfft layout (zeros outside the band)."""
    nl = band_shape_of(ub, Nx, Ns)
    shape = (nl, Ns, Nx // 2 + 1) if ub.dim() == 3 else (Ns, Nx // 2 + 1)
    uhat = torch.empty(shape, dtype=torch.complex128, device=ub.device)
    check(_lib.lib().loop_from_band(Nx, Ns, nl, _ptr(ub), _ptr(uhat), _stream_ptr()), "loop_from_band")
    return uhat


def _layout_of(u: torch.Tensor, layout: int, grid):
    if layout == LAYOUT_RFFT:
        return shape_of(u)
    Nx, Ns = grid
    return band_shape_of(u, Nx, Ns), int(Nx), int(Ns)


def saved_u(nloops: int, Nx: int, Ns: int, device) -> torch.Tensor:
    """An empty buffer for the forward's u on the s grid (nloops, C, Ns) complex128, the
    `usave` of loop_cost_fwd / loop_cost_bwd."""
    C, _ = band_dims(Nx, Ns)
    return torch.empty((nloops, C, Ns), dtype=torch.complex128, device=device)


def _check_usave(usave, nl, Nx, Ns, device):
    if usave is None:
        return None
    C, _ = band_dims(Nx, Ns)
    if (usave.shape != (nl, C, Ns) or usave.dtype != torch.complex128 or not usave.is_contiguous()
            or usave.device != device):
        raise ValueError(f"usave must be a contiguous complex128 tensor of shape {(nl, C, Ns)} on {device}")
    return _ptr(usave)


def loop_cost_fwd(u: torch.Tensor, T, L: float, layout: int = LAYOUT_RFFT, grid=None, ws: Workspace = None,
                  usave: torch.Tensor = None):
    """Forward pass of the cost: (J, dJ/dT, rsave), rsave the band residual the reverse pass
    takes. `grid` = (Nx, Ns) for the band layout. usave (see saved_u), if given, receives u on
    the s grid for the reverse pass."""
    nl, Nx, Ns = _layout_of(u, layout, grid)
    T = _periods(T, nl, u.device)
    C, NB = band_dims(Nx, Ns)
    J = torch.empty(nl, dtype=torch.float64, device=u.device)
    dJdT = torch.empty(nl, dtype=torch.float64, device=u.device)
    rsave = torch.empty((nl, C, NB), dtype=torch.complex128, device=u.device)
    us = _check_usave(usave, nl, Nx, Ns, u.device)
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_cost_fwd(float(L), Nx, Ns, nl, int(layout), _ptr(T), _ptr(u), _ptr(J), _ptr(dJdT),
                                   _ptr(rsave), us, ws.ptr, ws.nbytes, _stream_ptr()), "loop_cost_fwd")
    return J, dJdT, rsave


def loop_cost_bwd(u: torch.Tensor, T, L: float, rsave: torch.Tensor, dJdT: torch.Tensor, gJ: torch.Tensor = None,
                  layout: int = LAYOUT_RFFT, grid=None, ws: Workspace = None, usave: torch.Tensor = None):
    """Reverse pass from the forward's saved residual: (grad_u, grad_T) of sum_l gJ[l] J_l.
    usave: the buffer the forward of the same u filled, or None to recompute u on the grid."""
    nl, Nx, Ns = _layout_of(u, layout, grid)
    T = _periods(T, nl, u.device)
    if gJ is not None and (gJ.dtype != torch.float64 or gJ.numel() != nl or not gJ.is_contiguous()):
        raise ValueError("gJ must be a contiguous float64 tensor with one entry per loop")
    us = _check_usave(usave, nl, Nx, Ns, u.device)
    gu = torch.empty_like(u)
    gT = torch.empty(nl, dtype=torch.float64, device=u.device)
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_cost_bwd(float(L), Nx, Ns, nl, int(layout), _ptr(T), _ptr(u), _ptr(rsave), us,
                                   _ptr(dJdT), _ptr(gJ) if gJ is not None else None, _ptr(gu), _ptr(gT), ws.ptr,
                                   ws.nbytes, _stream_ptr()), "loop_cost_bwd")
    return gu, gT


def loop_update_grad(u: torch.Tensor, T: torch.Tensor, L: float, grad_u: torch.Tensor, grad_T: torch.Tensor,
                     dtau: float, scheme: int = EXPLICIT, layout: int = LAYOUT_RFFT, grid=None):
    """In place: the step of Sec. 4.2 from the gradient of sum_l J_l (G_1 = -grad_u / (w_j L))."""
    nl, Nx, Ns = _layout_of(u, layout, grid)
    T = _periods(T, nl, u.device)
    if grad_u.shape != u.shape or grad_u.dtype != u.dtype or not grad_u.is_contiguous():
        raise ValueError("grad_u must match u")
    grad_T = _periods(grad_T, nl, u.device)
    check(_lib.lib().loop_update_grad(float(L), Nx, Ns, nl, int(layout), _ptr(T), _ptr(u), _ptr(grad_u), _ptr(grad_T),
                                      float(dtau), int(scheme), _stream_ptr()), "loop_update_grad")
    return u, T


def loop_step(uhat: torch.Tensor, T: torch.Tensor, L: float, dtau: float, scheme: int = EXPLICIT,
              nsteps: int = 1, J_hist: torch.Tensor = None, ws: Workspace = None):
    """Advance (uhat, T) in place by nsteps. J_hist, if given, is float64 (nsteps, nloops)."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    if J_hist is not None and (J_hist.dtype != torch.float64 or J_hist.numel() < nsteps * nl
                               or not J_hist.is_contiguous()):
        raise ValueError("J_hist must be a contiguous float64 tensor with nsteps * nloops entries")
    ws = ws or workspace(Nx, Ns, nl)
    jh = _ptr(J_hist) if J_hist is not None else None
    check(_lib.lib().loop_step(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), float(dtau), int(scheme), int(nsteps),
                               jh, ws.ptr, ws.nbytes, _stream_ptr()), "loop_step")
    return uhat, T


def loop_extrapolate(uhat: torch.Tensor, T: torch.Tensor, uhat_a: torch.Tensor, T_a: torch.Tensor,
                     factor: torch.Tensor):
    """In place: (uhat, T) <- (uhat, T) + factor * ((uhat, T) - (uhat_a, T_a)), per loop (App. C)."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    T_a = _periods(T_a, nl, uhat.device)
    if uhat_a.shape != uhat.shape or uhat_a.dtype != uhat.dtype or not uhat_a.is_contiguous():
        raise ValueError("uhat_a must match uhat")
    factor = factor.to(device=uhat.device, dtype=torch.float64).contiguous()
    if factor.numel() != nl:
        raise ValueError("factor needs one entry per loop")
    check(_lib.lib().loop_extrapolate(Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(T_a), _ptr(uhat_a), _ptr(factor),
                                      _stream_ptr()), "loop_extrapolate")
    return uhat, T


def loop_converge(uhat: torch.Tensor, T: torch.Tensor, L: float, dtau: float, scheme: int, J_tol: float,
                  stride: int = 100, max_steps: int = 10 ** 7, accelerate: bool = True, sqrtJ_first: float = 1e-3,
                  ws: Workspace = None) -> dict:
    """Advance the loops in place until J < J_tol (see loop_converge in the C header), with or
    without the extrapolations of App. C. Returns per-loop steps (-1: not converged),
    extrapolations and final J."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    ws = ws or workspace(Nx, Ns, nl)
    steps = (ctypes.c_longlong * nl)()
    ext = (ctypes.c_int * nl)()
    Jf = (ctypes.c_double * nl)()
    check(_lib.lib().loop_converge(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), float(dtau), int(scheme), float(J_tol),
                                   int(stride), int(max_steps), 1 if accelerate else 0, float(sqrtJ_first), steps, ext,
                                   Jf, ws.ptr, ws.nbytes, _stream_ptr()), "loop_converge")
    return {"steps": list(steps), "extrapolations": list(ext), "J": list(Jf)}


RESIDENT_NEVER, RESIDENT_AUTO, RESIDENT_ALWAYS = 0, 1, 2


def set_resident(mode: int) -> int:
    """Choose the form of loop_step for later calls: RESIDENT_NEVER (per-pass kernels),
    RESIDENT_AUTO (the default: resident where measured faster) or RESIDENT_ALWAYS (resident
    wherever the loop fits in LDS). Returns the previous mode."""
    prev = _lib.lib().loop_set_resident(int(mode))
    if prev < 0:
        check(prev, "loop_set_resident")
    return prev


def step_form(Nx: int, Ns: int, nloops: int = 1) -> str:
    """"resident" or "per-pass": the form loop_step takes for these loops under the current mode."""
    f = _lib.lib().loop_step_form(int(Nx), int(Ns), int(nloops))
    if f < 0:
        check(f, "loop_step_form")
    return "resident" if f == 1 else "per-pass"


def resident_supported(Nx: int, Ns: int) -> bool:
    """Whether loop_step takes an Nx x Ns loop in the LDS-resident form on this device."""
    return bool(_lib.lib().loop_resident_supported(int(Nx), int(Ns)))


def loop_step_xi(uhat: torch.Tensor, T: torch.Tensor, L: float, dtau: float, scheme: int = EXPLICIT,
                 nsteps: int = 1, J_hist: torch.Tensor = None, ws: Workspace = None):
    """loop_step for centre-symmetric loops (u odd in x), in place, with half the state and
    traffic. The input is projected onto centre-symmetric loops first."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    if J_hist is not None and (J_hist.dtype != torch.float64 or J_hist.numel() < nsteps * nl
                               or not J_hist.is_contiguous()):
        raise ValueError("J_hist must be a contiguous float64 tensor with nsteps * nloops entries")
    ws = ws or workspace(Nx, Ns, nl)
    jh = _ptr(J_hist) if J_hist is not None else None
    check(_lib.lib().loop_step_xi(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), float(dtau), int(scheme), int(nsteps),
                                  jh, ws.ptr, ws.nbytes, _stream_ptr()), "loop_step_xi")
    return uhat, T


def loop_expanded_grad(uhat: torch.Tensor, T, L: float, ws: Workspace = None):
    """The paper's expanded form of the flow (eq. KS_G_1): (G1_hat, dJ/dT, J), as
    loop_adjoint_grad returns them."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    G = torch.empty_like(uhat)
    dT = torch.empty(nl, dtype=torch.float64, device=uhat.device)
    J = torch.empty(nl, dtype=torch.float64, device=uhat.device)
    ws = ws or workspace(Nx, Ns, nl)
    check(_lib.lib().loop_expanded_grad(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(G), _ptr(dT), _ptr(J), ws.ptr,
                                        ws.nbytes, _stream_ptr()), "loop_expanded_grad")
    return G, dT, J


def loop_step_expanded(uhat: torch.Tensor, T: torch.Tensor, L: float, dtau: float, scheme: int = EXPLICIT,
                       nsteps: int = 1, J_hist: torch.Tensor = None, ws: Workspace = None):
    """The paper's step on the expanded form (Sec. 4.2), in place, as loop_step."""
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    if J_hist is not None and (J_hist.dtype != torch.float64 or J_hist.numel() < nsteps * nl
                               or not J_hist.is_contiguous()):
        raise ValueError("J_hist must be a contiguous float64 tensor with nsteps * nloops entries")
    ws = ws or workspace(Nx, Ns, nl)
    jh = _ptr(J_hist) if J_hist is not None else None
    check(_lib.lib().loop_step_expanded(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), float(dtau), int(scheme),
                                        int(nsteps), jh, ws.ptr, ws.nbytes, _stream_ptr()), "loop_step_expanded")
    return uhat, T


def xi_workspace_bytes(Nx: int, Ns: int, nloops: int = 1) -> int:
    b = ctypes.c_size_t(0)
    check(_lib.lib().loop_step_xi_workspace_bytes(int(Nx), int(Ns), int(nloops), ctypes.byref(b)),
          "loop_step_xi_workspace_bytes")
    return int(b.value)


def loop_update(uhat: torch.Tensor, T: torch.Tensor, L: float, Ghat: torch.Tensor, dJdT: torch.Tensor,
                dtau: float, scheme: int = EXPLICIT):
    nl, Nx, Ns = shape_of(uhat)
    T = _periods(T, nl, uhat.device)
    check(_lib.lib().loop_update(float(L), Nx, Ns, nl, _ptr(T), _ptr(uhat), _ptr(Ghat), _ptr(dJdT), float(dtau),
                                 int(scheme), _stream_ptr()), "loop_update")
    return uhat, T


class Batch:
    """Loops of uneven (L, Nx, Ns) advanced together by the batched kernels.

    The spectra live back to back in one complex128 pool (rfft layout per loop, in the order
    given); `offsets[l]` is loop l's first element. The plan's device tables and the work
    space are allocated here, once, so that `step` can be captured into a graph.
    """

    def __init__(self, shapes, device=None):
        self.shapes = [(float(L), int(Nx), int(Ns)) for (L, Nx, Ns) in shapes]
        n = len(self.shapes)
        Ls = (ctypes.c_double * n)(*[s[0] for s in self.shapes])
        Nxs = (ctypes.c_int * n)(*[s[1] for s in self.shapes])
        Nss = (ctypes.c_int * n)(*[s[2] for s in self.shapes])
        plan = ctypes.c_void_p()
        check(_lib.lib().loop_batch_create(n, Ls, Nxs, Nss, ctypes.byref(plan)), "loop_batch_create")
        self._plan = plan
        wsb, pe = ctypes.c_size_t(0), ctypes.c_size_t(0)
        offs = (ctypes.c_longlong * n)()
        check(_lib.lib().loop_batch_info(plan, ctypes.byref(wsb), ctypes.byref(pe), offs), "loop_batch_info")
        self.pool_elems = int(pe.value)
        self.offsets = [int(o) for o in offs]
        self.nloops = n
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.ws = torch.empty(max(int(wsb.value), 256), dtype=torch.uint8, device=device)
        check(_lib.lib().loop_batch_workspace_init(plan, _ptr(self.ws), self.ws.numel(), _stream_ptr()),
              "loop_batch_workspace_init")

    PER_PASS = 0
    PERSISTENT = 1
    STREAMS = 2

    def set_schedule(self, schedule: int, nstreams: int = None):
        """PER_PASS (four launches per step), PERSISTENT (one launch for all steps) or STREAMS
        (the loops in nstreams groups, 2 to 4, on as many streams, one pass apart)."""
        check(_lib.lib().loop_batch_set_schedule(self._plan, int(schedule)), "loop_batch_set_schedule")
        if nstreams is not None:
            check(_lib.lib().loop_batch_set_streams(self._plan, int(nstreams)), "loop_batch_set_streams")

    def set_wait_limit(self, seconds: float):
        """Bound of one dependency wait of the persistent schedule (see loop_batch_set_wait_limit)."""
        check(_lib.lib().loop_batch_set_wait_limit(self._plan, float(seconds)), "loop_batch_set_wait_limit")

    VARIANTS = 4
    PASS_NAMES = ("A", "B", "C", "D", "E")

    def set_variant(self, pass_id: int, variant: int):
        """Kernel variant of one pass of the per-pass schedule (see loop_batch_set_variant)."""
        check(_lib.lib().loop_batch_set_variant(self._plan, int(pass_id), int(variant)), "loop_batch_set_variant")

    def config(self) -> dict:
        """The schedule and the kernel variant of each pass currently in use."""
        sc, ns = ctypes.c_int(0), ctypes.c_int(0)
        v = (ctypes.c_int * 5)()
        check(_lib.lib().loop_batch_get_config(self._plan, ctypes.byref(sc), v, ctypes.byref(ns)),
              "loop_batch_get_config")
        name = ("per-pass", "persistent", f"streams-{ns.value}")[sc.value]
        return {"schedule": name, "variants": {n: int(v[i]) for i, n in enumerate(self.PASS_NAMES)}}

    def autotune(self, pool, T, reps=20) -> dict:
        """Time every usable kernel variant of every pass, then the per-pass and the streams
        schedules, on this state (pool and T are left unchanged) and keep the fastest (see
        loop_batch_autotune; the persistent schedule is not timed). Returns the timings in
        microseconds and the chosen configuration."""
        self._check_state(pool, T)
        n = 5 * self.VARIANTS + 5
        rep = (ctypes.c_double * n)()
        check(_lib.lib().loop_batch_autotune(self._plan, _ptr(T), _ptr(pool), int(reps), rep, _ptr(self.ws),
                                             self.ws.numel(), _stream_ptr()),
              "loop_batch_autotune")
        passes = {}
        for i, name in enumerate(self.PASS_NAMES):
            passes[name] = {v: round(rep[i * self.VARIANTS + v], 3) for v in range(self.VARIANTS)
                            if rep[i * self.VARIANTS + v] >= 0}
        out = self.config()
        out["pass_us"] = passes
        names = ("per-pass", "persistent", "streams-2", "streams-3", "streams-4")
        out["step_us"] = {name: round(rep[5 * self.VARIANTS + i], 3) for i, name in enumerate(names)
                          if rep[5 * self.VARIANTS + i] >= 0}
        return out

    def _check_state(self, pool, T):
        if pool.dtype != torch.complex128 or pool.numel() != self.pool_elems or not pool.is_contiguous():
            raise ValueError("pool must be the contiguous complex128 pool of this plan")
        if T.dtype != torch.float64 or T.numel() != self.nloops or not T.is_contiguous():
            raise ValueError("T must be float64 with one entry per loop")

    def pack(self, spectra):
        """Pool tensor holding the given per-loop spectra (each (Ns, Nx//2+1) complex128)."""
        dev = self.ws.device
        pool = torch.zeros(self.pool_elems, dtype=torch.complex128, device=dev)
        for (L, Nx, Ns), off, u in zip(self.shapes, self.offsets, spectra):
            u = torch.as_tensor(u).to(dev).reshape(-1)
            if u.numel() != Ns * (Nx // 2 + 1):
                raise ValueError("spectrum shape does not match the plan")
            pool[off:off + u.numel()] = u
        return pool

    def unpack(self, pool):
        """Views of the pool, one (Ns, Nx//2+1) tensor per loop."""
        return [pool[off:off + Ns * (Nx // 2 + 1)].view(Ns, Nx // 2 + 1)
                for (L, Nx, Ns), off in zip(self.shapes, self.offsets)]

    def step(self, pool, T, dtau, scheme=EXPLICIT, nsteps=1, J_hist=None):
        self._check_state(pool, T)
        if J_hist is not None and (J_hist.dtype != torch.float64 or J_hist.numel() < nsteps * self.nloops):
            raise ValueError("J_hist must be float64 (nsteps, nloops)")
        jh = _ptr(J_hist) if J_hist is not None else None
        check(_lib.lib().loop_batch_step(self._plan, _ptr(T), _ptr(pool), float(dtau), int(scheme), int(nsteps), jh,
                                         _ptr(self.ws), self.ws.numel(), _stream_ptr()), "loop_batch_step")
        return pool, T

    def load(self, pool):
        check(_lib.lib().loop_batch_load(self._plan, _ptr(pool), _ptr(self.ws), self.ws.numel(), _stream_ptr()),
              "loop_batch_load")

    def run_pass(self, pass_id, step, nsteps, T, dtau, scheme=EXPLICIT, J_hist=None):
        jh = _ptr(J_hist) if J_hist is not None else None
        check(_lib.lib().loop_batch_pass(self._plan, int(pass_id), int(step), int(nsteps), _ptr(T), float(dtau),
                                         int(scheme), jh, _ptr(self.ws), self.ws.numel(), _stream_ptr()),
              "loop_batch_pass")

    def store(self, pool):
        check(_lib.lib().loop_batch_store(self._plan, _ptr(pool), _ptr(self.ws), self.ws.numel(), _stream_ptr()),
              "loop_batch_store")

    def status(self) -> int:
        return int(_lib.lib().loop_status_sync(_ptr(self.ws), _stream_ptr()))

    def reset(self):
        """Prepare the work space again (clears the sticky status and the schedule counters)."""
        check(_lib.lib().loop_batch_workspace_init(self._plan, _ptr(self.ws), self.ws.numel(), _stream_ptr()),
              "loop_batch_workspace_init")

    def __del__(self):
        try:
            if getattr(self, "_plan", None) is not None and self._plan.value:
                _lib.lib().loop_batch_destroy(self._plan)
                self._plan = None
        except Exception:
            pass


class trace:
    """Kernel timing by HIP events that each library launch's dispatch records at its kernel's
    start and end (see loop_trace_start):

        with api.trace() as tr:
            ...                       # library calls
        tr.kernels                    # {name: {"launches", "total_us", "avg_us", "min_us", "max_us"}}
    """

    def __enter__(self):
        check(_lib.lib().loop_trace_start(), "loop_trace_start")
        self.kernels = {}
        return self

    def __exit__(self, *exc):
        check(_lib.lib().loop_trace_stop(), "loop_trace_stop")
        L = _lib.lib()
        buf = ctypes.create_string_buffer(128)
        n, tot, lo, hi = ctypes.c_longlong(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        for i in range(L.loop_trace_count()):
            check(L.loop_trace_get(i, buf, 128, ctypes.byref(n), ctypes.byref(tot), ctypes.byref(lo), ctypes.byref(hi)),
                  "loop_trace_get")
            self.kernels[buf.value.decode()] = {"launches": int(n.value), "total_us": tot.value,
                                                "avg_us": tot.value / max(n.value, 1), "min_us": lo.value,
                                                "max_us": hi.value}
        return False
