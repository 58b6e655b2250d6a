"""Throughput benchmark of the KS loop-space adjoint step on one MI355X.

A step is one pass of the whole hot path over every loop of the workload. That pass covers
the residual r, the cost J, dJ/dT, the adjoint flow G and the fictitious-time update of
(u_hat, T). Inputs are seeded synthetic loops, already resident in HBM when the timed region
starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched-256x1024",
                    choices=["batched-256x1024", "plain-64x128", "plain-32x32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return ap.parse_args()


WORKLOAD_CFG = {"plain-32x32": 1, "plain-64x128": 2, "batched-256x1024": 5}


def algorithmic_bytes_per_step(Nx, Ns, nloops):
    """HBM bytes one step must move in the four-kernel schedule (complex values are 16 B).

    Intermediates A, B, C, D of (Kx+1) x Ns complex values: A is written once and read twice
    (passes B and D), B, C and D are written once and read once. That gives 9 W. Band state
    traffic: u_hat is read in pass C, U1 = u_hat + dtau sigma G_lin is written in C and read in
    E, and u_hat' is written in E. That gives 4 S, with S = (Kx+1)(2Ks+1) band values.
    """
    Kx, Ks = (Nx - 1) // 3, (Ns - 1) // 3
    W = (Kx + 1) * Ns
    S = (Kx + 1) * (2 * Ks + 1)
    return 16 * (9 * W + 4 * S) * nloops


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import loopgen
    from paper_2007_06427_amd import api

    c = WORKLOAD_CFG[args.workload]
    cfg = loopgen.CONFIGS[c]
    steps = args.steps if args.steps is not None else min(cfg["steps"], 2000)
    specs = loopgen.config_loops(c)
    Nx, Ns, L = specs[0].Nx, specs[0].Ns, specs[0].L
    nl = len(specs)
    scheme = api.IMEX if cfg["scheme"] == "imex" else api.EXPLICIT
    dtau = cfg["dtau"]

    torch.cuda.set_device(0)
    api.init()
    u0 = torch.from_numpy(np.stack([s.uhat for s in specs])).to("cuda:0")
    T0 = torch.tensor([s.T for s in specs], dtype=torch.float64, device="cuda:0")
    u = u0.clone()
    T = T0.clone()
    ws = api.workspace(Nx, Ns, nl)
    stream = torch.cuda.current_stream()

    # warm-up
    api.loop_step(u, T, L, dtau, scheme, args.warmup, ws=ws)
    torch.cuda.synchronize()
    assert ws.status() == 0

    # timed region: `steps` steps in one loop_step call, bracketed by events on its stream
    Jh = torch.zeros(steps, nl, dtype=torch.float64, device="cuda:0")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    api.loop_step(u, T, L, dtau, scheme, steps, J_hist=Jh, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert ws.status() == 0, "device flagged a non-finite state"
    gpu_s = e0.elapsed_time(e1) / 1e3
    pts = Nx * Ns * nl * steps
    value = pts / wall
    J = Jh.cpu().numpy()
    assert np.all(np.isfinite(J))

    bytes_step = algorithmic_bytes_per_step(Nx, Ns, nl)
    step_avg = gpu_s / steps
    achieved = bytes_step / step_avg / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "one step (four kernels: B, C, D, E+A)", "bytes_per_launch": bytes_step}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(specs, dtau, scheme)

    out = {
        "metric": "space-time pts/s of r+J+adjoint G+update (FP64)",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": nl, "Nx": Nx, "Ns": Ns, "L": L,
                   "scheme": cfg["scheme"], "dtau": dtau, "parallelism": "none (1 GPU)"},
        "roofline": roofline, "cpu_baseline": cpu,
        "J_first_last": [float(J[0].mean()), float(J[-1].mean())],
    }
    print(json.dumps(out))


def cpu_baseline(specs, dtau, scheme):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    from oracle import ks_loop as K
    threads = int(os.environ.get("OMP_NUM_THREADS", "1") or 1)
    s = specs[0]
    t0 = time.perf_counter()
    n = 0
    u, T = s.uhat, s.T
    while time.perf_counter() - t0 < 10.0 and n < 2000:
        u, T, _ = K.step(u, T, s.L, dtau, scheme, 1)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": s.Nx * s.Ns * n / dt, "unit": "pts/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of loop 0 ({s.Nx}x{s.Ns}), single process"}


if __name__ == "__main__":
    main()
