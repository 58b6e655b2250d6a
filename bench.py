"""Throughput benchmark of the KS loop-space adjoint step on one MI355X.

A step is one pass of the whole hot path over every loop of the workload: the residual r,
the cost J, dJ/dT, the adjoint flow G and the fictitious-time update of (u_hat, T). Inputs
are seeded synthetic loops, already resident in HBM when the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Workloads:
  batched-ragged-256  (default) 256 loops, Nx in {32, 64}, Ns in {64..512}, L in {22, 39}, IMEX
  batched-256x1024    64 loops of 256 x 1024, L = 100, IMEX
  plain-64x128        one 64 x 128 loop, L = 22, IMEX
  plain-32x32         one 32 x 32 loop, L = 22, explicit Euler

Prints one JSON line. `value` counts space-time points (sum over loops of Nx * Ns) advanced
per second of wall time over K steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PASS_NAMES = {1: "B (rows: u u_x)", 2: "C (columns: residual, J, dJ/dT)", 3: "D (rows: u r_x, period)",
              4: "E (columns: G and update, next A)"}
KERNEL_OF_PASS = {1: "k_rag<1>", 2: "k_rag<2>", 3: "k_rag<3>", 4: "k_rag<4>"}

WORKLOADS = {
    "batched-ragged-256": 4,
    "batched-256x1024": 5,
    "plain-64x128": 2,
    "plain-32x32": 1,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched-ragged-256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return ap.parse_args()


def band(Nx, Ns):
    C = (Nx - 1) // 3 + 1
    NB = 2 * ((Ns - 1) // 3) + 1
    return C * Ns, C * NB  # W (intermediate column values), S (band values)


def pass_bytes(shapes, p):
    """Algorithmic HBM bytes of one launch of pass p over all loops (16 B per complex value).

    B reads A and writes B (2W). C reads B and u_hat and writes C and U1 (2W + 2S). D reads A
    and C and writes D (3W). E reads D and U1 and writes u_hat' and the next A (2W + 2S).
    A step moves 9W + 4S.
    """
    tot = 0
    for (Nx, Ns) in shapes:
        W, S = band(Nx, Ns)
        tot += {1: 2 * W, 2: 2 * W + 2 * S, 3: 3 * W, 4: 2 * W + 2 * S}[p]
    return 16 * tot


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken on this source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    from paper_2007_06427_amd.profiling import source_digest
    d = json.load(open(path))
    if d.get("source_digest") != source_digest():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import loopgen
    from paper_2007_06427_amd import api

    c = WORKLOADS[args.workload]
    cfg = loopgen.CONFIGS[c]
    steps = args.steps if args.steps is not None else cfg["steps"]
    specs = loopgen.config_loops(c)
    shapes = [(s.Nx, s.Ns) for s in specs]
    nl = len(specs)
    pts_step = sum(Nx * Ns for Nx, Ns in shapes)
    scheme = api.IMEX if cfg["scheme"] == "imex" else api.EXPLICIT
    dtau = cfg["dtau"]

    torch.cuda.set_device(0)
    api.init()
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    batch = api.Batch([(s.L, s.Nx, s.Ns) for s in specs])
    pool0 = batch.pack([torch.from_numpy(s.uhat) for s in specs])
    T0 = torch.tensor([s.T for s in specs], dtype=torch.float64, device=dev)

    # ---- warm-up
    pool, T = pool0.clone(), T0.clone()
    batch.step(pool, T, dtau, scheme, args.warmup)
    torch.cuda.synchronize()
    assert batch.status() == 0

    # ---- timed region: K steps, one loop_batch_step call (per-pass schedule)
    pool, T = pool0.clone(), T0.clone()
    Jh = torch.zeros(steps, nl, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    batch.step(pool, T, dtau, scheme, steps, J_hist=Jh)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert batch.status() == 0, "device flagged a non-finite state"
    J = Jh.cpu().numpy()
    assert np.all(np.isfinite(J))
    value = pts_step * steps / wall

    # ---- per-kernel timing of the same step, pass by pass, with events on the launch stream.
    # A backlog of queued steps keeps the GPU busy while the host enqueues the instrumented
    # launches, so that no event pair includes host launch latency.
    Kr = min(steps, 100)
    step_s = wall / steps
    pb, Tb = pool0.clone(), T0.clone()
    batch.step(pb, Tb, dtau, scheme, max(20, int(0.05 / step_s)))
    pool, T = pool0.clone(), T0.clone()
    batch.load(pool)
    batch.run_pass(0, 0, Kr, T, dtau, scheme)
    evs = {p: [] for p in (1, 2, 3, 4)}
    for s in range(Kr):
        for p in (1, 2, 3, 4):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            batch.run_pass(p, s, Kr, T, dtau, scheme)
            b.record(stream)
            evs[p].append((a, b))
    batch.store(pool)
    torch.cuda.synchronize()
    assert batch.status() == 0
    avg_us = {p: 1e3 * sum(a.elapsed_time(b) for a, b in v) / len(v) for p, v in evs.items()}
    passes_sum_us = sum(avg_us.values())
    dom = max(avg_us, key=lambda p: avg_us[p])
    by = pass_bytes(shapes, dom)
    achieved = by / (avg_us[dom] * 1e-6) / 1e9
    traffic = measured_traffic(args.workload, KERNEL_OF_PASS[dom])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"{KERNEL_OF_PASS[dom]} pass {PASS_NAMES[dom]}", "bytes_per_launch": by,
                "avg_launch_us": round(avg_us[dom], 2),
                "passes_us": {KERNEL_OF_PASS[p]: round(v, 2) for p, v in avg_us.items()},
                "passes_sum_vs_step": round(passes_sum_us / (step_s * 1e6), 3),
                "step_bytes": sum(pass_bytes(shapes, p) for p in (1, 2, 3, 4))}

    # ---- plain method on the same loops: loop_step per loop, one after another
    plain = None
    if nl > 1:
        Kp = 10
        sub = []
        for s in specs:
            u = torch.from_numpy(s.uhat[None]).to(dev)
            Tl = torch.tensor([s.T], dtype=torch.float64, device=dev)
            sub.append((u, Tl, s.L, api.Workspace(api.workspace_bytes(s.Nx, s.Ns, 1))))
        for (u, Tl, L, ws) in sub:
            api.loop_step(u, Tl, L, dtau, scheme, 1, ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for (u, Tl, L, ws) in sub:
            api.loop_step(u, Tl, L, dtau, scheme, Kp, ws=ws)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t1
        plain = {"value": pts_step * Kp / tp, "unit": "pts/s", "steps": Kp,
                 "method": "loop_step per loop, sequential on one stream"}

    # a plain device copy of known size: its counter readings calibrate FETCH_SIZE / WRITE_SIZE
    src = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()

    cpu = None if args.no_cpu else cpu_baseline(specs, dtau, scheme)

    out = {
        "metric": "space-time pts/s of r+J+adjoint G+update (FP64)",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": nl, "shapes": sorted(set(shapes)),
                   "scheme": cfg["scheme"], "dtau": dtau, "schedule": "per-pass launches",
                   "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": e0.elapsed_time(e1) / steps,
        "roofline": roofline, "cpu_baseline": cpu, "plain": plain,
        "batched_vs_plain": (value / plain["value"]) if plain else None,
        "J_first_last": [float(J[0].mean()), float(J[-1].mean())],
    }
    print(json.dumps(out))


def cpu_baseline(specs, dtau, scheme, budget_s=15.0):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same workload: whole
    steps of the workload's loops in order, until the time budget is spent."""
    from oracle import ks_loop as K
    threads = 1  # numpy.fft (pocketfft) runs each transform on one thread
    t0 = time.perf_counter()
    pts = 0
    done = 0
    steps_each = 4 if len(specs) > 1 else 10 ** 9
    for s in specs:
        u, T = s.uhat, s.T
        n = 0
        while n < steps_each and time.perf_counter() - t0 < budget_s:
            u, T, _ = K.step(u, T, s.L, dtau, scheme, 1)
            pts += s.Nx * s.Ns
            n += 1
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": pts / dt, "unit": "pts/s", "cores": threads, "kind": "oracle",
            "sample": f"{pts} space-time points: up to {steps_each} steps each of the first {done} loops "
                      "(NumPy FP64, one process, one thread)"}


if __name__ == "__main__":
    main()
