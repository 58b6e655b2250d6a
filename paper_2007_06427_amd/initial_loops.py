"""Tensor-level binding of the initial-loop pipeline (include/ks_initial_loops.h, Sec. 4.3):
chaotic KS runs, recurrences of their norm and the temporal low-pass that makes loops.

Instantaneous states are complex128 device tensors of shape (ntraj, Nx//2 + 1) in the rfft
layout; loops come out in the layout of the loop dynamics, (nloops, Ns, Nx//2 + 1), with their
periods. Torch provides device memory and streams only; the arithmetic runs in
liblooporbit.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import check
from .api import _ptr, _stream_ptr


def _states(uhat: torch.Tensor):
    if uhat.dtype != torch.complex128 or not uhat.is_cuda or not uhat.is_contiguous() or uhat.dim() != 2:
        raise ValueError("states must be a contiguous complex128 device tensor (ntraj, Nx//2 + 1)")
    return int(uhat.shape[0]), 2 * (int(uhat.shape[1]) - 1)


def _offset(t: Optional[torch.Tensor], elems: int):
    """Device pointer to element `elems` of t (None for no tensor)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr() + elems * t.element_size())


def ks_integrate(uhat: torch.Tensor, L: float, dt: float, nsteps: int, sample_every: int = 1,
                 symmetric: bool = False, norms: Optional[torch.Tensor] = None,
                 snaps: Optional[torch.Tensor] = None, first_sample: int = 0):
    """Advance the runs `uhat` (in place) by nsteps ETDRK4 steps. Samples of the states before
    steps 0, s, 2s, ... go to norms[:, first_sample + i] (float64, (ntraj, stride)) and
    snaps[:, first_sample + i] (complex128, (ntraj, stride, Nx//2 + 1)) when given."""
    ntraj, Nx = _states(uhat)
    stride = 0
    for t, dt_, shape in ((norms, torch.float64, (ntraj,)), (snaps, torch.complex128, (ntraj,))):
        if t is None:
            continue
        if t.dtype != dt_ or not t.is_cuda or not t.is_contiguous() or tuple(t.shape[:1]) != shape:
            raise ValueError("norms / snaps must be contiguous device tensors with one row per run")
        stride = int(t.shape[1])
    if norms is not None and snaps is not None and norms.shape[1] != snaps.shape[1]:
        raise ValueError("norms and snaps must have the same number of samples per run")
    if snaps is not None and snaps.shape[2] != Nx // 2 + 1:
        raise ValueError("snaps must hold rows of Nx//2 + 1 values")
    ns = nsteps // sample_every if sample_every > 0 else 0
    if (norms is not None or snaps is not None) and not 0 <= first_sample <= stride - ns:
        raise ValueError("the samples of this call do not fit after first_sample")
    H = Nx // 2 + 1
    check(_lib.lib().ks_integrate(float(L), Nx, ntraj, 1 if symmetric else 0, float(dt), int(nsteps),
                                  int(sample_every), _ptr(uhat), _offset(norms, first_sample),
                                  _offset(snaps, first_sample * H), stride, _stream_ptr()), "ks_integrate")
    return uhat


def ks_recurrences(norms: torch.Tensor, nsamples: int, dt_s: float, rel_tol: float, Tmin: float, Tmax: float,
                   cap: int = 64):
    """Pairs of nearly equal maxima of each run's norm: (pairs (ntraj, cap, 2) int32 of sample
    indices (a, b), counts (ntraj,) int32; the first min(count, cap) pairs are valid)."""
    if norms.dtype != torch.float64 or not norms.is_cuda or not norms.is_contiguous() or norms.dim() != 2:
        raise ValueError("norms must be a contiguous float64 device tensor (ntraj, stride)")
    ntraj = int(norms.shape[0])
    pairs = torch.full((ntraj, max(cap, 1), 2), -1, dtype=torch.int32, device=norms.device)
    counts = torch.zeros(ntraj, dtype=torch.int32, device=norms.device)
    check(_lib.lib().ks_recurrences(ntraj, int(nsamples), _ptr(norms), int(norms.shape[1]), float(dt_s),
                                    float(rel_tol), float(Tmin), float(Tmax), int(cap), _ptr(pairs), _ptr(counts),
                                    _stream_ptr()), "ks_recurrences")
    return pairs[:, :cap], counts


def ks_segments_to_loops(snaps: torch.Tensor, nsamples: int, triples: torch.Tensor, dt_s: float, Ns: int, kc: int):
    """Loops of the segments triples[l] = (run, a, b): (uhat (nloops, Ns, Nx//2 + 1), T (nloops,))."""
    if snaps.dtype != torch.complex128 or not snaps.is_cuda or not snaps.is_contiguous() or snaps.dim() != 3:
        raise ValueError("snaps must be a contiguous complex128 device tensor (ntraj, stride, Nx//2 + 1)")
    if triples.dtype != torch.int32 or not triples.is_cuda or triples.dim() != 2 or triples.shape[1] != 3:
        raise ValueError("triples must be an int32 device tensor (nloops, 3)")
    triples = triples.contiguous()
    ntraj, stride, H = (int(d) for d in snaps.shape)
    nl = int(triples.shape[0])
    loops = torch.empty(nl, Ns, H, dtype=torch.complex128, device=snaps.device)
    T = torch.empty(nl, dtype=torch.float64, device=snaps.device)
    check(_lib.lib().ks_segments_to_loops(2 * (H - 1), ntraj, int(nsamples), _ptr(snaps), stride, nl, _ptr(triples),
                                          float(dt_s), int(Ns), int(kc), _ptr(loops), _ptr(T), _stream_ptr()),
          "ks_segments_to_loops")
    return loops, T


def initial_loops(u0: torch.Tensor, L: float, dt: float, n_transient: int, n_record: int, sample_every: int,
                  rel_tol: float, Tmin: float, Tmax: float, Ns: int, kc: int, symmetric: bool = True,
                  per_run: int = 4, cap: int = 256):
    """The whole pipeline of Sec. 4.3 on the runs u0 (advanced in place): n_transient steps
    unrecorded, n_record steps sampled every `sample_every`, recurrence pairs of the norm, and
    the first `per_run` pairs of each run (in order of their first maximum) made into loops.
    Returns (loops, T, triples, norms, snaps)."""
    ntraj, Nx = _states(u0)
    if n_transient:
        ks_integrate(u0, L, dt, n_transient, n_transient, symmetric)
    ns = n_record // sample_every
    norms = torch.empty(ntraj, ns, dtype=torch.float64, device=u0.device)
    snaps = torch.empty(ntraj, ns, Nx // 2 + 1, dtype=torch.complex128, device=u0.device)
    ks_integrate(u0, L, dt, n_record, sample_every, symmetric, norms, snaps)
    dt_s = dt * sample_every
    pairs, counts = ks_recurrences(norms, ns, dt_s, rel_tol, Tmin, Tmax, cap)
    take = torch.clamp(counts, max=min(per_run, cap)).cpu()
    pairs_h = pairs.cpu()
    rows = [(r, int(pairs_h[r, p, 0]), int(pairs_h[r, p, 1])) for r in range(ntraj) for p in range(int(take[r]))]
    if not rows:
        empty = torch.empty(0, Ns, Nx // 2 + 1, dtype=torch.complex128, device=u0.device)
        return empty, torch.empty(0, dtype=torch.float64, device=u0.device), torch.empty(0, 3, dtype=torch.int32), \
            norms, snaps
    triples = torch.tensor(rows, dtype=torch.int32).to(u0.device)
    loops, T = ks_segments_to_loops(snaps, ns, triples, dt_s, Ns, kc)
    return loops, T, triples, norms, snaps
