"""Host-only checks of the C-ABI library: it loads, exports every declared symbol, and rejects
bad arguments on the host before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2007_06427_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("looporbit.h", "ks_initial_loops.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b((?:loop|ks)_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_every_header_is_listed():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == sorted(os.path.basename(h) for h in HEADERS)


def test_header_declares_what_the_binding_binds():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    syms = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", syms), name


def test_status_strings():
    assert _lib.status_string(0) == "ok"
    assert "invalid" in _lib.status_string(_lib.LOOP_EINVAL)
    assert "unknown" in _lib.status_string(12345)


@pytest.mark.parametrize("Nx,Ns,nl,expect", [
    (48, 32, 1, _lib.LOOP_ENOTSUP), (32, 96, 1, _lib.LOOP_ENOTSUP), (4, 32, 1, _lib.LOOP_EINVAL),
    (32, 2048, 1, _lib.LOOP_EINVAL), (32, 32, 0, _lib.LOOP_EINVAL), (32, 32, -3, _lib.LOOP_EINVAL),
])
def test_workspace_bytes_rejects_bad_sizes(Nx, Ns, nl, expect):
    n = ctypes.c_size_t(0)
    assert _lib.lib().loop_workspace_bytes(Nx, Ns, nl, ctypes.byref(n)) == expect


def test_workspace_bytes_scales_with_batch():
    L = _lib.lib()
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.loop_workspace_bytes(64, 128, 1, ctypes.byref(a)) == 0
    assert L.loop_workspace_bytes(64, 128, 8, ctypes.byref(b)) == 0
    C = 64 // 3 + 1
    assert a.value >= 3 * 128 * C * 16  # three intermediates of N x C complex values
    assert 7 * a.value < b.value < 9 * a.value
    assert L.loop_workspace_bytes(64, 128, 1, None) == _lib.LOOP_EINVAL


def test_entry_points_reject_bad_arguments_on_host():
    L = _lib.lib()
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced: checks fail before any GPU work
    odd = ctypes.c_void_p((1 << 20) + 8)
    ws = ctypes.c_void_p(1 << 24)
    # null and misaligned pointers
    assert L.loop_residual(22.0, 32, 32, 1, None, fake, fake, ws, 1 << 30, None) == _lib.LOOP_EINVAL
    assert L.loop_residual(22.0, 32, 32, 1, fake, odd, ctypes.c_void_p(1 << 21), ws, 1 << 30, None) == _lib.LOOP_EINVAL
    # aliasing output and input
    assert L.loop_residual(22.0, 32, 32, 1, fake, fake, fake, ws, 1 << 30, None) == _lib.LOOP_EINVAL
    # bad L, sizes
    out = ctypes.c_void_p(1 << 21)
    assert L.loop_cost(0.0, 32, 32, 1, fake, fake, out, ws, 1 << 30, None) == _lib.LOOP_EINVAL
    assert L.loop_cost(float("nan"), 32, 32, 1, fake, fake, out, ws, 1 << 30, None) == _lib.LOOP_EINVAL
    assert L.loop_cost(22.0, 48, 32, 1, fake, fake, out, ws, 1 << 30, None) == _lib.LOOP_ENOTSUP
    # work space too small
    assert L.loop_cost(22.0, 32, 32, 1, fake, fake, out, ws, 1024, None) == _lib.LOOP_EWORKSPACE
    # misaligned work space
    assert L.loop_cost(22.0, 32, 32, 1, fake, fake, out, ctypes.c_void_p((1 << 24) + 64), 1 << 30, None) \
        == _lib.LOOP_EINVAL
    # bad step arguments
    for dtau, scheme, n in [(0.0, 0, 1), (-1e-4, 0, 1), (float("inf"), 0, 1), (1e-4, 2, 1), (1e-4, 0, -1)]:
        assert L.loop_step(22.0, 32, 32, 1, fake, fake, dtau, scheme, n, None, ws, 1 << 30, None) == _lib.LOOP_EINVAL
    assert L.loop_update(22.0, 32, 32, 1, fake, fake, out, fake, 0.0, 0, None) == _lib.LOOP_EINVAL
    assert L.loop_update(22.0, 32, 32, 1, fake, fake, fake, fake, 1e-4, 0, None) == _lib.LOOP_EINVAL
    assert L.loop_workspace_init(None, 1024, None) == _lib.LOOP_EINVAL
    assert L.loop_status_sync(odd, None) == _lib.LOOP_EINVAL


def test_reverse_mode_entry_points_reject_bad_arguments_on_host():
    L = _lib.lib()
    fake, fake2, fake3 = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), ctypes.c_void_p(1 << 22)
    odd = ctypes.c_void_p((1 << 20) + 8)
    ws = ctypes.c_void_p(1 << 24)
    E, W = _lib.LOOP_EINVAL, _lib.LOOP_EWORKSPACE
    band, rfft = _lib.LAYOUT_BAND, _lib.LAYOUT_RFFT
    fake4 = ctypes.c_void_p(1 << 23)
    fwd = L.loop_cost_fwd
    assert fwd(22.0, 32, 32, 1, 7, fake, fake, fake2, None, fake3, None, ws, 1 << 30, None) == E  # layout
    assert fwd(22.0, 32, 32, 1, rfft, fake, odd, fake2, None, fake3, None, ws, 1 << 30, None) == E  # misaligned u
    assert fwd(22.0, 32, 32, 1, band, fake, fake3, fake2, None, fake3, None, ws, 1 << 30, None) == E  # rsave = u
    assert fwd(22.0, 32, 32, 1, band, fake, fake, fake2, None, fake3, fake3, ws, 1 << 30, None) == E  # usave = rsave
    assert fwd(22.0, 32, 32, 1, band, fake, fake, fake2, None, fake3, fake, ws, 1 << 30, None) == E  # usave = u
    assert fwd(22.0, 32, 32, 1, band, fake, fake, fake2, None, fake3, odd, ws, 1 << 30, None) == E  # misaligned
    assert fwd(22.0, 32, 32, 1, band, fake, fake, fake2, None, fake3, None, ws, 1024, None) == W
    assert fwd(22.0, 32, 32, 1, band, fake, fake, fake2, None, fake3, fake4, ws, 1024, None) == W
    bwd = L.loop_cost_bwd
    assert bwd(22.0, 32, 32, 1, rfft, fake, fake, fake2, None, fake, None, fake, None, ws, 1 << 30, None) == E  # grad = u
    assert bwd(22.0, 32, 32, 1, rfft, fake, fake, fake2, None, fake, None, fake2, None, ws, 1 << 30, None) == E  # = rsave
    assert bwd(22.0, 32, 32, 1, rfft, fake, fake, fake2, fake4, fake, None, fake4, None, ws, 1 << 30, None) == E  # = usave
    assert bwd(22.0, 32, 32, 1, rfft, fake, fake, fake2, odd, fake, None, fake3, None, ws, 1 << 30, None) == E  # usave
    bad8 = ctypes.c_void_p((1 << 20) + 4)
    assert bwd(22.0, 32, 32, 1, band, fake, fake, fake2, None, bad8, None, fake3, fake, ws, 1 << 30, None) == E  # dJdT
    upd = L.loop_update_grad
    assert upd(22.0, 32, 32, 1, band, fake, fake2, fake2, fake, 1e-4, 1, None) == E  # grad aliases u
    assert upd(22.0, 32, 32, 1, band, fake, fake2, fake3, fake, 0.0, 1, None) == E  # dtau
    assert upd(22.0, 32, 32, 1, 3, fake, fake2, fake3, fake, 1e-4, 1, None) == E  # layout
    assert L.loop_to_band(32, 32, 1, fake, fake, None) == E
    assert L.loop_from_band(48, 32, 1, fake, fake2, None) == _lib.LOOP_ENOTSUP


def test_trace_outside_a_session_reports_nothing():
    L = _lib.lib()
    assert L.loop_trace_start() == 0 and L.loop_trace_stop() == 0
    assert L.loop_trace_count() == 0
    buf = ctypes.create_string_buffer(16)
    assert L.loop_trace_get(0, buf, 16, None, None, None, None) == _lib.LOOP_EINVAL


def test_initial_loop_entry_points_reject_bad_arguments_on_host():
    L = _lib.lib()
    fake = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 8)
    E, N = _lib.LOOP_EINVAL, _lib.LOOP_ENOTSUP
    ok = (39.0, 64, 4, 1, 0.05, 40, 4, fake, fake, fake, 10, None)

    def integ(**kw):
        names = ["L", "Nx", "ntraj", "sym", "dt", "nsteps", "every", "u", "norms", "snaps", "stride", "stream"]
        args = dict(zip(names, ok))
        args.update(kw)
        return L.ks_integrate(*[args[n] for n in names])
    for kw, want in [({"L": 0.0}, E), ({"dt": float("nan")}, E), ({"Nx": 512}, N), ({"Nx": 48}, N),
                     ({"Nx": 4}, E), ({"ntraj": 0}, E), ({"nsteps": -4}, E), ({"every": 0}, E),
                     ({"nsteps": 42}, E), ({"stride": 9}, E), ({"u": odd}, E), ({"u": None}, E),
                     ({"snaps": odd}, E)]:
        assert integ(**kw) == want, kw
    pairs, counts = ctypes.c_void_p(1 << 21), ctypes.c_void_p(1 << 22)
    rec = L.ks_recurrences
    assert rec(0, 10, fake, 10, 0.1, 0.01, 1.0, 5.0, 4, pairs, counts, None) == E
    assert rec(2, 10, fake, 9, 0.1, 0.01, 1.0, 5.0, 4, pairs, counts, None) == E
    assert rec(2, 10, fake, 10, 0.0, 0.01, 1.0, 5.0, 4, pairs, counts, None) == E
    assert rec(2, 10, fake, 10, 0.1, -0.01, 1.0, 5.0, 4, pairs, counts, None) == E
    assert rec(2, 10, fake, 10, 0.1, 0.01, float("nan"), 5.0, 4, pairs, counts, None) == E
    assert rec(2, 10, fake, 10, 0.1, 0.01, 1.0, 5.0, 4, None, counts, None) == E
    assert rec(2, 10, ctypes.c_void_p((1 << 20) + 4), 10, 0.1, 0.01, 1.0, 5.0, 4, pairs, counts, None) == E
    seg = L.ks_segments_to_loops
    assert seg(48, 2, 10, fake, 10, 1, fake, 0.1, 64, 5, fake, fake, None) == E
    assert seg(64, 2, 10, fake, 10, 1, fake, 0.1, 64, 22, fake, fake, None) == E
    assert seg(64, 2, 10, fake, 10, 0, fake, 0.1, 64, 5, fake, fake, None) == E
    assert seg(64, 2, 10, fake, 9, 1, fake, 0.1, 64, 5, fake, fake, None) == E
    assert seg(64, 2, 10, odd, 10, 1, fake, 0.1, 64, 5, fake, fake, None) == E
    assert seg(64, 2, 10, fake, 10, 1, fake, 0.0, 64, 5, fake, fake, None) == E
