"""Host checks of bench.py: its one-GPU contract and its byte model.

The byte model (16 B per complex value; per loop and step 9W + 4S, with W = (Kx+1) Ns column
values and S = (Kx+1)(2Ks+1) band values) is checked against the oracle's band mask and against
the HBM traffic the hardware counters measured for each pass (profiles/traffic_*.json)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import loopgen
from oracle import ks_loop as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    d = json.loads(p.stdout.strip().splitlines()[-1])
    assert d["n_gpus"] == 2 and "one GPU" in d["error"]


@pytest.mark.parametrize("Nx,Ns", [(8, 8), (32, 64), (64, 512), (256, 1024), (1024, 16)])
def test_band_sizes_follow_the_oracles_band(Nx, Ns):
    W, S = bench.band(Nx, Ns)
    mask = K.band_mask(Nx, Ns)  # (Ns, Nx/2 + 1) rfft layout, j >= 0
    assert S == int(mask.sum())
    assert W == int(mask.any(axis=0).sum()) * Ns  # band columns, each of Ns values


def test_passes_add_up_to_the_step_model():
    for Nx, Ns in [(32, 64), (64, 512), (256, 1024)]:
        W, S = bench.band(Nx, Ns)
        assert sum(bench.pass_bytes([(Nx, Ns)], p) for p in (1, 2, 3, 4)) == 16 * (9 * W + 4 * S)


@pytest.mark.parametrize("workload", ["batched-ragged-256", "batched-256x1024"])
def test_byte_model_agrees_with_the_measured_traffic(workload):
    """Every pass moves, by FETCH_SIZE + WRITE_SIZE (calibrated by a device copy), within 5% of
    its algorithmic bytes: no pass re-reads what it has read. The ragged workload fits in the
    Infinity Cache; the 64 loops of 256 x 1024 do not."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    d = json.load(open(path))
    # the calibration dispatch is the 64 MiB copy: WRITE_SIZE counts its 65536 KiB exactly
    assert abs(d["copy_calibration"]["write_kib"] - 65536.0) < 1.0
    shapes = [(s.Nx, s.Ns) for s in loopgen.config_loops(bench.WORKLOADS[workload])]
    seen = 0
    for name, k in d["kernels"].items():
        if not name.startswith("k_rag<") or name.startswith("k_rag<0"):
            continue  # pass A (k_rag<0, v>) also converts the caller's layout; it runs once per call
        p = int(name[len("k_rag<"):].split(",")[0])
        alg = bench.pass_bytes(shapes, p)
        assert abs(k["bytes_per_launch"] / alg - 1.0) < 0.05, (name, k["bytes_per_launch"], alg)
        seen += 1
    assert seen >= 4


def test_flop_model_counts_every_transform():
    """step_flops is 5 n log2 n per n-point complex transform: 4 per band column of Ns points,
    3 per row pair of Nx points over two row passes (B and D each hold two inverse and one
    forward transform per pair of rows, Ns/2 pairs), plus the pointwise work."""
    Nx, Ns = 64, 128
    C = K.band_limits(Nx, Ns)[0] + 1
    transforms = 4 * C * 5 * Ns * np.log2(Ns) + 2 * (Ns // 2) * 3 * 5 * Nx * np.log2(Nx)
    pointwise = bench.step_flops(Nx, Ns) - transforms
    assert 0 < pointwise < 0.2 * bench.step_flops(Nx, Ns)


def test_autograd_kernels_add_up_to_their_step_model():
    """The seven kernels of an autograd-path step move 16 (10W + 10S) bytes per loop."""
    for Nx, Ns in [(64, 256), (256, 1024)]:
        W, S = bench.band(Nx, Ns)
        kb = bench.autograd_kernel_bytes(Nx, Ns)
        assert len(kb) == 7 and sum(kb.values()) == 16 * (10 * W + 10 * S)


def test_autograd_byte_model_agrees_with_the_measured_traffic():
    """Each kernel of the autograd step (launches over all 64 loops of 256 x 1024) moves, by
    FETCH_SIZE + WRITE_SIZE, within 5% of its algorithmic bytes (autograd_kernel_bytes), and
    the save_u path's k_colR too (16 (S + W) per loop)."""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_autograd-256x1024.json")))
    assert abs(d["copy_calibration"]["write_kib"] - 65536.0) < 1.0
    specs = loopgen.config_loops(bench.WORKLOADS["autograd-256x1024"])
    Nx, Ns, nl = specs[0].Nx, specs[0].Ns, len(specs)
    W, S = bench.band(Nx, Ns)
    want = {k: v * nl for k, v in bench.autograd_kernel_bytes(Nx, Ns).items()}
    want[f"k_colR<{Ns}>"] = 16 * (S + W) * nl
    for name, alg in want.items():
        got = d["kernels"][name]["bytes_per_launch"]
        assert abs(got / alg - 1.0) < 0.05, (name, got, alg)
