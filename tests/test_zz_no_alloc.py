"""loop_step_noalloc: loop_step with the library's static device work space instead of a
caller-owned one (for callers that cannot allocate). It runs loop_step's kernels, so its results
must equal loop_step's bit for bit, call after call, whatever the previous call left in the
shared array."""
import ctypes

import numpy as np
import pytest

import loopgen
from paper_2007_06427_amd import _lib

SCRATCH_BYTES = 64 << 20  # LOOP_NOALLOC_SCRATCH_BYTES


def _loops(seed, nloops, Nx, Ns, L):
    specs = [loopgen.random_loop(100 * seed + i, L, Nx, Ns, min(8, Nx // 3), min(8, Ns // 3), 0.5, 0.2, (30.0, 60.0))
             for i in range(nloops)]
    return np.stack([s.uhat for s in specs]), np.array([s.T for s in specs])


def test_noalloc_rejects_shapes_beyond_its_array():
    L = _lib.lib()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the size check fails first
    need = ctypes.c_size_t(0)
    assert L.loop_workspace_bytes(256, 1024, 20, ctypes.byref(need)) == 0
    assert need.value > SCRATCH_BYTES
    assert L.loop_step_noalloc(100.0, 256, 1024, 20, fake, fake, 5e-5, 1, 1, None, None, None) == _lib.LOOP_EWORKSPACE
    # the usual argument checks come first
    assert L.loop_step_noalloc(100.0, 256, 1024, 1, fake, fake, 0.0, 1, 1, None, None, None) == _lib.LOOP_EINVAL
    assert L.loop_step_noalloc(100.0, 48, 1024, 1, fake, fake, 5e-5, 1, 1, None, None, None) == _lib.LOOP_ENOTSUP
    assert L.loop_step_noalloc(100.0, 256, 1024, 1, fake, fake, 5e-5, 1, 1, None, ctypes.c_void_p((1 << 20) + 2),
                               None) == _lib.LOOP_EINVAL


@pytest.mark.gpu
def test_noalloc_equals_loop_step_call_after_call():
    import torch

    from paper_2007_06427_amd import api
    torch.cuda.set_device(0)
    api.init()
    L = _lib.lib()
    dev = "cuda:0"
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # a larger per-pass batch, then a smaller one, a resident loop, a non-finite period (the status
    # must say so, and the next call must start from a cleared status), and the first batch again
    cases = [(0, 4, 64, 256, 39.0, 1, 3), (1, 2, 32, 128, 22.0, 0, 2), (2, 1, 32, 32, 22.0, 0, 5),
             (3, 2, 32, 64, 22.0, 1, 1), (0, 4, 64, 256, 39.0, 1, 3)]
    for (seed, nl, Nx, Ns, Ld, scheme, nsteps) in cases:
        u0, T0 = _loops(seed, nl, Nx, Ns, Ld)
        bad = seed == 3
        if bad:
            T0[1] = -T0[1]
        print(f"noalloc case seed={seed} nloops={nl} {Nx}x{Ns} form={api.step_form(Nx, Ns, nl)}", flush=True)
        dtau = 5e-5 if scheme == 1 else 1e-5
        ua = torch.from_numpy(u0).to(dev)
        Ta = torch.from_numpy(T0).to(dev)
        ub, Tb = ua.clone(), Ta.clone()
        Ja = torch.zeros(nsteps, nl, dtype=torch.float64, device=dev)
        Jb = torch.zeros_like(Ja)
        status = torch.full((1,), 12345, dtype=torch.int32, device=dev)
        # reference: loop_step with a work space of its own
        ws = api.Workspace(api.workspace_bytes(Nx, Ns, nl))
        assert L.loop_step(Ld, Nx, Ns, nl, ctypes.c_void_p(Ta.data_ptr()), ctypes.c_void_p(ua.data_ptr()), dtau, scheme,
                           nsteps, ctypes.c_void_p(Ja.data_ptr()), ws.ptr, ws.nbytes, stream) == 0
        st_ref = ws.status()
        assert L.loop_step_noalloc(Ld, Nx, Ns, nl, ctypes.c_void_p(Tb.data_ptr()), ctypes.c_void_p(ub.data_ptr()), dtau,
                                   scheme, nsteps, ctypes.c_void_p(Jb.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                                   stream) == 0
        torch.cuda.synchronize()
        assert int(status.item()) == st_ref == (_lib.LOOP_ENONFINITE if bad else 0)
        if bad:
            continue
        assert torch.equal(ua, ub)
        assert torch.equal(Ta, Tb)
        assert torch.equal(Ja, Jb)
        assert np.all(np.isfinite(Jb.cpu().numpy()))
