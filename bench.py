"""Throughput benchmark of the KS loop-space adjoint step on one MI355X.

A step is one pass of the whole hot path over every loop of the workload: the residual r,
the cost J, dJ/dT, the adjoint flow G and the fictitious-time update of (u_hat, T). Inputs
are seeded synthetic loops, already resident in HBM when the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Workloads:
  autograd-256x1024   (default) 64 loops of 256 x 1024, L = 100, IMEX dtau = 5e-5, 2000 steps:
                      G from the autograd path (LoopCostBand forward and its adjoint backward)
                      and one fused update kernel (loop_update_grad); beside it the same path on
                      rfft-layout tensors, the fused batched step, the plain method and the oracle
  batched-256x1024    the same 64 loops, fused batched step (loop_batch_step) alone
  batched-ragged-256  256 loops, Nx in {32, 64}, Ns in {64..512}, L in {22, 39}, IMEX
  converge-32x32      the 32 x 32 loop driven to J < 1e-10 (IMEX, dtau = 0.05, J examined every
                      100 steps), with and without the extrapolations of App. C
  xi-256x1024         the same 64 loops projected onto centre-symmetric loops (u odd in x),
                      stepped by loop_step_xi (half the state), with loop_step on the same loops
                      beside it
  orbits-39           the initial-loop pipeline of Sec. 4.3 and the loop dynamics together:
                      128 centre-symmetric chaotic KS runs at L = 39 (64 modes, ETDRK4), their
                      norm recurrences with 20 <= T <= 160 made into 256 loops of 64 x 64, the
                      loops driven by loop_converge (IMEX, dtau = 0.15, App. C extrapolations);
                      reports the periods of the orbits found beside the paper's
  expanded-256x1024   the 64 loops of 256 x 1024 stepped by the paper's own expanded form of the
                      flow (eq. KS_G_1, loop_step_expanded), with loop_step beside it
  ks-dns-4096         the chaotic runs of the initial-loop pipeline alone: 4096 centre-symmetric
                      KS runs at L = 39 on 64 modes, ETDRK4 with dt = 0.05, sampled every 2 steps
  plain-64x128        one 64 x 128 loop, L = 22, IMEX dtau = 5e-5, 20 000 steps; logs J(tau) and
                      T(tau) every 10 steps
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

METRIC = "space-time pts/s of r+J+adjoint G (FP64); batched vs plain; HBM GB/s fraction"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
CUS = 256
PASS_NAMES = {1: "B (rows: u u_x)", 2: "C (columns: residual, J, dJ/dT)", 3: "D (rows: u r_x, period)",
              4: "E (columns: G and update, next A)"}

WORKLOADS = {
    "batched-ragged-256": 4,
    "batched-256x1024": 5,
    "autograd-256x1024": 5,
    "xi-256x1024": 5,
    "expanded-256x1024": 5,
    "plain-64x128": 2,
    "plain-32x32": 1,
    "converge-32x32": 1,
    "orbits-39": 1,
    "ks-dns-4096": 1,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="autograd-256x1024", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--runs", type=int, default=128, help="orbits-39: chaotic runs")
    ap.add_argument("--per-run", type=int, default=2, help="orbits-39: loops cut from each run")
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


def step_flops(Nx, Ns):
    """Algorithmic FP64 flops of one step of one loop (5 n log2 n per complex n-point transform):
    four transforms per band column (C: forward and inverse; E: forward and the next step's
    inverse), three per row over passes B and D (each pass: two inverse and one forward per
    pair of rows), about 55 per band value for the spectral assembly and update, and the
    physical-space products."""
    C = (Nx - 1) // 3 + 1
    S = C * (2 * ((Ns - 1) // 3) + 1)
    lg = lambda n: n.bit_length() - 1
    return 20 * C * Ns * lg(Ns) + 15 * Ns * Nx * lg(Nx) + 55 * S + 4 * Nx * Ns


def copy_ceiling_gbs(device, mib=512, reps=20):
    """Read plus write bandwidth of a plain device-to-device copy of `mib` MiB (larger than the
    256 MB Infinity Cache), timed between events over `reps` back-to-back copies: the practical
    streaming ceiling the kernels' HBM figures can be set against. Outside any timed region."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.empty(n, dtype=torch.float64, device=device).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 8 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


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
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}))
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
    # A plain device copy of known size, before any other copy of the run: its counter
    # readings calibrate FETCH_SIZE and WRITE_SIZE (the first large copy of a counter run).
    src = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    torch.empty_like(src).copy_(src)
    torch.cuda.synchronize()
    del src
    if args.workload.startswith("converge"):
        return bench_converge(args, specs[0])
    if args.workload.startswith("orbits"):
        return bench_orbits(args, E=args.runs, per_run=args.per_run)
    if args.workload.startswith("ks-dns"):
        return bench_dns(args)
    if nl == 1 and api.step_form(specs[0].Nx, specs[0].Ns, 1) == "resident":
        return bench_resident(args, cfg, specs[0], steps, dtau, scheme)
    if nl == 1:
        return bench_plain(args, cfg, specs[0], steps, dtau, scheme)
    if args.workload.startswith("autograd"):
        return bench_autograd(args, cfg, specs, steps, dtau, scheme)
    if args.workload.startswith("xi"):
        return bench_xi(args, cfg, specs, steps, dtau, scheme)
    if args.workload.startswith("expanded"):
        return bench_expanded(args, cfg, specs, steps, dtau, scheme)
    batch = api.Batch([(s.L, s.Nx, s.Ns) for s in specs])
    pool0 = batch.pack([torch.from_numpy(s.uhat) for s in specs])
    T0 = torch.tensor([s.T for s in specs], dtype=torch.float64, device=dev)

    # ---- kernel variants and schedule chosen by the autotuner (before any timed work)
    tuning = batch.autotune(pool0, T0, reps=20)
    torch.cuda.synchronize()
    variants = tuning["variants"]

    def kernel_of(p):
        return f"k_rag<{p}, {variants['ABCDE'[p]]}>"

    # ---- warm-up
    pool, T = pool0.clone(), T0.clone()
    batch.step(pool, T, dtau, scheme, args.warmup)
    torch.cuda.synchronize()
    assert batch.status() == 0

    # ---- timed region: K steps, one loop_batch_step call (the tuned schedule)
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

    # ---- per-kernel timing, pass by pass (each pass over every loop, alone on the stream, as
    # the per-pass schedule runs it), with events on the launch stream. Every pass is a
    # function of the work space alone, so pass p is launched R times back to back between one
    # event pair; the launches take a negligible step (a kernel's work does not depend on it),
    # so that pass D's repeated period updates leave T where it is. A backlog of queued whole
    # steps goes first, so that the GPU never waits on the host inside an event pair.
    R = 50
    step_s = wall / steps
    pool, T = pool0.clone(), T0.clone()
    nback = max(20, min(200, int(0.01 / step_s)))
    avg_us = {}
    for p in (1, 2, 3, 4):
        batch.step(pool, T, dtau, scheme, nback)
        batch.load(pool)
        batch.run_pass(0, 0, 2, T, dtau, scheme)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(R):
            batch.run_pass(p, 0, 2, T, 1e-30, scheme)  # step 0 of 2: E also forms the next A
        b.record(stream)
        torch.cuda.synchronize()
        avg_us[p] = 1e3 * a.elapsed_time(b) / R
    assert batch.status() == 0
    passes_sum_us = sum(avg_us.values())
    dom = max(avg_us, key=lambda p: avg_us[p])
    by = pass_bytes(shapes, dom)
    achieved = by / (avg_us[dom] * 1e-6) / 1e9
    traffic = measured_traffic(args.workload, kernel_of(dom))
    step_bytes = sum(pass_bytes(shapes, p) for p in (1, 2, 3, 4))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"{kernel_of(dom)} pass {PASS_NAMES[dom]}", "bytes_per_launch": by,
                "avg_launch_us": round(avg_us[dom], 2),
                "passes_us": {kernel_of(p): round(v, 2) for p, v in avg_us.items()},
                "passes_sum_vs_step": round(passes_sum_us / (step_s * 1e6), 3),
                "step_bytes": step_bytes,
                # the whole step, every pass, as the timed region ran it (its kernels may overlap)
                "step_achieved": round(step_bytes / (e0.elapsed_time(e1) * 1e-3 / steps) / 1e9, 1),
                "step_frac": round(step_bytes / (e0.elapsed_time(e1) * 1e-3 / steps) / 1e9 / HBM_PEAK_GBS, 4)}
    copy_gbs = copy_ceiling_gbs(dev)
    roofline["copy_gbs"] = round(copy_gbs, 1)  # plain 512 MiB device copy, same machine
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)

    # ---- context for the schedule choice (same loops, min(K, 500) steps each, not the headline):
    # all steps in one persistent launch, and the tuned schedule's steps recorded once into a
    # HIP graph and replayed
    kc = min(steps, 500)

    def gpu_ms_per_step(fn):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / kc

    def captured(step_call):
        """the call recorded once into a HIP graph (after one call off the graph)"""
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step_call(2)
        stream.wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step_call(kc)
        g.replay()
        return g

    tuned = batch.config()["schedule"]
    batch.set_schedule(api.Batch.PERSISTENT)
    pool, T = pool0.clone(), T0.clone()
    batch.step(pool, T, dtau, scheme, 2)
    persistent_ms = gpu_ms_per_step(lambda: batch.step(pool, T, dtau, scheme, kc))
    assert batch.status() == 0
    pool, T = pool0.clone(), T0.clone()
    persistent_graph = captured(lambda n: batch.step(pool, T, dtau, scheme, n))
    persistent_graph_ms = gpu_ms_per_step(persistent_graph.replay)
    assert batch.status() == 0 and bool(torch.isfinite(T).all())
    if tuned.startswith("streams"):
        batch.set_schedule(api.Batch.STREAMS, int(tuned.split("-")[1]))
    else:
        batch.set_schedule(api.Batch.PER_PASS)
    pool, T = pool0.clone(), T0.clone()
    graph = captured(lambda n: batch.step(pool, T, dtau, scheme, n))
    graph_ms = gpu_ms_per_step(graph.replay)
    assert batch.status() == 0 and bool(torch.isfinite(T).all())
    schedules = {"tuned": tuned, "steps": kc, "tuned_eager_ms_per_step": round(e0.elapsed_time(e1) / steps, 5),
                 "persistent_ms_per_step": round(persistent_ms, 5),
                 "persistent_graph_replay_ms_per_step": round(persistent_graph_ms, 5),
                 "tuned_graph_replay_ms_per_step": round(graph_ms, 5),
                 "method": "persistent: loop_batch_step with LOOP_BATCH_PERSISTENT, one launch for all steps, "
                           "eager and recorded into a HIP graph (torch.cuda.CUDAGraph) and replayed; graph: the "
                           "tuned schedule's loop_batch_step call of all steps recorded and replayed"}

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

    cpu = None if args.no_cpu else cpu_baseline(specs, dtau, scheme)
    cpu_all = None if args.no_cpu else cpu_baseline_all_cores(specs, dtau, scheme)

    out = {
        "metric": METRIC,
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": nl, "shapes": sorted(set(shapes)),
                   "scheme": cfg["scheme"], "dtau": dtau, "schedule": tuning["schedule"],
                   "variants": variants,
                   "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": e0.elapsed_time(e1) / steps,
        "roofline": roofline, "cpu_baseline": cpu, "cpu_baseline_all_cores": cpu_all, "plain": plain,
        "autotune": {"pass_us": tuning["pass_us"], "step_us": tuning["step_us"]},
        "schedules": schedules,
        "batched_vs_plain": (value / plain["value"]) if plain else None,
        "J_first_last": [float(J[0].mean()), float(J[-1].mean())],
    }
    print(json.dumps(out))


def bench_resident(args, cfg, spec, steps, dtau, scheme):
    """One loop through loop_step, which takes it in the LDS-resident form: one block, every
    step in a single launch. That kernel is bound by FP64 arithmetic and LDS latency on the one
    CU it occupies, so its roofline is FP64 flops against the vector peak (and per CU used)."""
    import numpy as np
    import torch

    from paper_2007_06427_amd import api
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    u0 = torch.from_numpy(spec.uhat[None]).to(dev)
    T0 = torch.tensor([spec.T], dtype=torch.float64, device=dev)
    ws = api.Workspace(api.workspace_bytes(spec.Nx, spec.Ns, 1))
    u, T = u0.clone(), T0.clone()
    api.loop_step(u, T, spec.L, dtau, scheme, args.warmup, ws=ws)
    torch.cuda.synchronize()
    assert ws.status() == 0
    u, T = u0.clone(), T0.clone()
    Jh = torch.zeros(steps, 1, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    api.loop_step(u, T, spec.L, dtau, scheme, steps, J_hist=Jh, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert ws.status() == 0, "device flagged a non-finite state"
    J = Jh.cpu().numpy()[:, 0]
    assert np.all(np.isfinite(J))
    pts = spec.Nx * spec.Ns
    gpu_s = e0.elapsed_time(e1) * 1e-3
    fl = step_flops(spec.Nx, spec.Ns)
    achieved = fl * steps / gpu_s / 1e12
    cpu = None if args.no_cpu else cpu_baseline([spec], dtau, scheme)
    out = {
        "metric": METRIC,
        "value": pts * steps / wall, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": 1, "shapes": [[spec.Nx, spec.Ns]], "scheme": cfg["scheme"],
                   "dtau": dtau, "form": "resident (one block, all steps in one launch)",
                   "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": gpu_s / steps * 1e3,
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 6), "traffic": None,
                     "kernel": f"k_resident<{spec.Nx}, {spec.Ns}>", "flops_per_step": fl,
                     "avg_launch_us": round(gpu_s * 1e6, 1), "cus_used": 1,
                     "frac_of_cus_used": round(achieved / (FP64_PEAK_TFLOPS / CUS), 4)},
        "cpu_baseline": cpu,
        "J_first_last": [float(J[0]), float(J[-1])],
    }
    print(json.dumps(out))


def bench_plain(args, cfg, spec, steps, dtau, scheme, every=10):
    """One loop through loop_step in the per-pass form: K steps in one call (the timed region),
    then the log the workload asks for, J(tau) and T(tau) every `every` steps, from a run of the
    same steps in calls of `every` steps. Each call first makes the state canonical (column 0
    exactly Hermitian), which the steps inside one call keep only to rounding, so the two runs
    agree to rounding; their largest relative difference in J is reported."""
    import numpy as np
    import torch

    from paper_2007_06427_amd import api
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    u0 = torch.from_numpy(spec.uhat[None]).to(dev)
    T0 = torch.tensor([spec.T], dtype=torch.float64, device=dev)
    ws = api.Workspace(api.workspace_bytes(spec.Nx, spec.Ns, 1))
    u, T = u0.clone(), T0.clone()
    api.loop_step(u, T, spec.L, dtau, scheme, args.warmup, ws=ws)
    torch.cuda.synchronize()
    u, T = u0.clone(), T0.clone()
    Jh = torch.zeros(steps, 1, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    api.loop_step(u, T, spec.L, dtau, scheme, steps, J_hist=Jh, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert ws.status() == 0, "device flagged a non-finite state"
    J = Jh.cpu().numpy()[:, 0]
    assert np.all(np.isfinite(J))
    # the log: T at the start of every `every`-th step, J at the same steps
    n = steps // every
    u2, T2 = u0.clone(), T0.clone()
    Jh2 = torch.zeros_like(Jh)
    Tl = torch.zeros(n, dtype=torch.float64, device=dev)
    with api.trace() as tr:
        for i in range(n):
            Tl[i].copy_(T2[0])
            api.loop_step(u2, T2, spec.L, dtau, scheme, every, J_hist=Jh2[i * every:(i + 1) * every], ws=ws)
    J2 = Jh2.cpu().numpy()[:, 0]
    dev_rel = float(np.max(np.abs(J2 - J) / np.abs(J)))
    assert dev_rel < 1e-10, "the logged run left the timed run's trajectory"
    kb = {f"k_rowB<{spec.Nx}>": pass_bytes([(spec.Nx, spec.Ns)], 1),
          f"k_colC<{spec.Ns}, 3>": pass_bytes([(spec.Nx, spec.Ns)], 2),
          f"k_rowD<{spec.Nx}>": pass_bytes([(spec.Nx, spec.Ns)], 3),
          f"k_colE<{spec.Ns}, 3>": pass_bytes([(spec.Nx, spec.Ns)], 4)}
    kern = {k: v for k, v in tr.kernels.items() if k in kb}
    dom = max(kern, key=lambda k: kern[k]["total_us"])
    achieved = kb[dom] / (kern[dom]["avg_us"] * 1e-6) / 1e9
    gpu_s = e0.elapsed_time(e1) * 1e-3
    pts = spec.Nx * spec.Ns
    cpu = None if args.no_cpu else cpu_baseline([spec], dtau, scheme)
    out = {
        "metric": METRIC,
        "value": pts * steps / wall, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": 1, "shapes": [[spec.Nx, spec.Ns]], "L": spec.L,
                   "scheme": cfg["scheme"], "dtau": dtau, "form": "per-pass (loop_step)", "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": gpu_s / steps * 1e3,
        # one loop spreads a pass over a few blocks: latency-bound, far from the HBM roofline
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None, "kernel": dom,
                     "bytes_per_launch": kb[dom], "avg_launch_us": round(kern[dom]["avg_us"], 2),
                     "kernels_us": {k: round(v["avg_us"], 2) for k, v in tr.kernels.items()}},
        "cpu_baseline": cpu,
        "log_every": every,
        "logged_vs_timed_J_max_rel": dev_rel,
        "J_log": [float(f"{x:.12g}") for x in J2[::every]],
        "T_log": [float(f"{x:.12g}") for x in Tl.cpu().numpy()],
        "J_final": float(api.loop_cost(u, T, spec.L).item()), "T_final": float(T.item()),
    }
    print(json.dumps(out))


def autograd_kernel_bytes(Nx, Ns):
    """Algorithmic HBM bytes of each kernel of one autograd-path step of one loop, band layout
    (16 B per complex value; W = C Ns values of one transform intermediate, S = C NB band values):
      forward  k_colA  reads u_hat, writes A                 S + W
               k_rowB  reads A, writes B                     2W
               k_colC  reads B and u_hat, writes r_hat       W + 2S
      backward k_colAC reads u_hat and r_hat, writes A, C    2S + 2W
               k_rowD  reads A and C, writes D               3W
               k_colE  reads D and r_hat, writes the grad    W + 2S
      update   k_update_grad_band reads u_hat, grad; writes u_hat   3S
    16 (10W + 10S) per loop-step; the per-loop scalars (J, dJ/dT, T) are left out. (With u on the
    s grid kept from the forward, k_colR reads r_hat and writes C alone: 16 (9W + 9S).)"""
    W, S = band(Nx, Ns)
    return {f"k_colA<{Ns}>": 16 * (S + W), f"k_rowB<{Nx}>": 16 * 2 * W, f"k_colC<{Ns}, 0>": 16 * (W + 2 * S),
            f"k_colAC<{Ns}>": 16 * (2 * S + 2 * W), f"k_rowD<{Nx}>": 16 * 3 * W, f"k_colE<{Ns}, 4>": 16 * (W + 2 * S),
            "k_update_grad_band": 16 * 3 * S}


def bench_autograd(args, cfg, specs, steps, dtau, scheme):
    """The large batched workload as specified: per step, J = LoopCostBand(u_hat, T) forward,
    J.backward() through the hand-written adjoint kernels (which recompute the transform
    intermediates instead of storing them), and one fused update kernel
    (loop_update_grad) that takes the gradient: G_1 = -grad / (w_j L), the IMEX step of u_hat and
    the explicit step of T. The state is held in the band layout (the retained modes); the
    conversion from and to the rfft layout is inside the timed region, once. Beside it: the same
    path on rfft-layout tensors (LoopCost), the band path that keeps u on the s grid (save_u),
    the fused batched step (loop_batch_step, tuned) and the plain method (loop_step per loop), all
    on the same loops, and the CPU oracle."""
    import numpy as np
    import torch

    from paper_2007_06427_amd import api, autograd
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    L = specs[0].L
    Nx, Ns = specs[0].Nx, specs[0].Ns
    nl = len(specs)
    assert all((s.L, s.Nx, s.Ns) == (L, Nx, Ns) for s in specs)
    grid = (Nx, Ns)
    u0 = torch.from_numpy(np.stack([s.uhat for s in specs])).to(dev)
    T0 = torch.tensor([s.T for s in specs], dtype=torch.float64, device=dev)
    ones = torch.ones(nl, dtype=torch.float64, device=dev)
    ws = api.workspace(Nx, Ns, nl)

    def run_band(ub, T, k, save_u=False):
        for _ in range(k):
            ua = ub.detach().requires_grad_(True)
            Ta = T.detach().requires_grad_(True)
            autograd.LoopCostBand.apply(ua, Ta, L, Nx, Ns, save_u).backward(ones)
            api.loop_update_grad(ub, T, L, ua.grad, Ta.grad, dtau, scheme, layout=api.LAYOUT_BAND, grid=grid)

    def run_rfft(u, T, k):
        for _ in range(k):
            ua = u.detach().requires_grad_(True)
            Ta = T.detach().requires_grad_(True)
            autograd.LoopCost.apply(ua, Ta, L).backward(ones)
            api.loop_update_grad(u, T, L, ua.grad, Ta.grad, dtau, scheme)

    def timed(fn, k):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        out = fn(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3, out

    def band_path(k):
        ub, T = api.to_band(u0), T0.clone()
        run_band(ub, T, k)
        return api.from_band(ub, Nx, Ns), T

    def rfft_path(k):
        u, T = u0.clone(), T0.clone()
        run_rfft(u, T, k)
        return u, T

    # ---- warm-up, then the timed region: K steps of the band-layout autograd path
    band_path(args.warmup)
    assert ws.status() == 0
    wall, gpu_s, (u_ag, T_ag) = timed(band_path, steps)
    assert ws.status() == 0, "device flagged a non-finite state"
    J_end = api.loop_cost(u_ag, T_ag, L).cpu().numpy()
    assert np.all(np.isfinite(J_end)) and bool(torch.all(T_ag > 0))
    pts_step = Nx * Ns * nl
    value = pts_step * steps / wall

    # ---- per-kernel durations: HIP events around every launch on its stream, over a run of the
    # same call sequence (kept apart from the timed region so that it runs undisturbed)
    kb = autograd_kernel_bytes(Nx, Ns)
    ktrace = min(steps, 50)
    ub, T = api.to_band(u0), T0.clone()
    run_band(ub, T, 2)
    torch.cuda.synchronize()
    with api.trace() as tr:
        run_band(ub, T, ktrace)
    kern = {k: v for k, v in tr.kernels.items() if k in kb}
    dom = max(kern, key=lambda k: kern[k]["total_us"])
    by = kb[dom] * nl
    achieved = by / (kern[dom]["avg_us"] * 1e-6) / 1e9
    step_bytes = sum(kb.values()) * nl
    traced_step_us = sum(v["total_us"] for v in tr.kernels.values()) / ktrace
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, dom),
                "kernel": dom, "bytes_per_launch": by, "avg_launch_us": round(kern[dom]["avg_us"], 2),
                "byte_model": "16 (10W + 10S) B per loop-step over seven kernels (W = C Ns, S = C NB)",
                "kernels_us": {k: round(v["avg_us"], 2) for k, v in tr.kernels.items()},
                "kernels_frac": {k: round(kb[k] * nl / (v["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                 for k, v in kern.items()},
                "step_bytes": step_bytes,
                "step_achieved": round(step_bytes / (gpu_s / steps) / 1e9, 1),
                "step_frac": round(step_bytes / (gpu_s / steps) / 1e9 / HBM_PEAK_GBS, 4),
                "traced_kernels_sum_vs_step": round(traced_step_us / (gpu_s / steps * 1e6), 3)}
    copy_gbs = copy_ceiling_gbs(dev)
    roofline["copy_gbs"] = round(copy_gbs, 1)  # plain 512 MiB device copy, same machine
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)
    roofline["step_frac_of_copy"] = round(step_bytes / (gpu_s / steps) / 1e9 / copy_gbs, 4)

    # ---- the same path on rfft-layout tensors
    k_r = min(steps, 200)
    rfft_path(min(args.warmup, 5))
    wall_r, gpu_r, (u_r, T_r) = timed(rfft_path, k_r)

    # ---- the band path with u on the s grid kept from the forward (save_u): one column
    # transform fewer in the backward, a grid-sized saved tensor
    def band_saved(k):
        ub, T = api.to_band(u0), T0.clone()
        run_band(ub, T, k, save_u=True)
        return api.from_band(ub, Nx, Ns), T
    band_saved(min(args.warmup, 5))
    wall_n, gpu_n, (u_n, _) = timed(band_saved, k_r)
    if k_r == steps:  # the same steps: the same state, bit for bit
        assert torch.equal(u_n, u_ag)

    # ---- the fused batched step on the same loops (tuned), K steps
    batch = api.Batch([(s.L, s.Nx, s.Ns) for s in specs])
    pool0 = batch.pack([torch.from_numpy(s.uhat) for s in specs])
    tuning = batch.autotune(pool0, T0, reps=10)
    pool, Tf = pool0.clone(), T0.clone()
    batch.step(pool, Tf, dtau, scheme, args.warmup)
    torch.cuda.synchronize()

    def fused(k):
        pool, Tf = pool0.clone(), T0.clone()
        batch.step(pool, Tf, dtau, scheme, k)
        return pool, Tf
    wall_f, gpu_f, (pool_f, T_f) = timed(fused, steps)
    assert batch.status() == 0
    u_f = torch.stack(batch.unpack(pool_f))
    diff = float(np.max(np.abs(u_f.cpu().numpy() - u_ag.cpu().numpy())) / np.max(np.abs(u_f.cpu().numpy())))

    # ---- plain method on the same loops: loop_step per loop, one after another
    Kp = 10
    sub = []
    for s_ in specs:
        u = torch.from_numpy(s_.uhat[None]).to(dev)
        Tl = torch.tensor([s_.T], dtype=torch.float64, device=dev)
        sub.append((u, Tl, api.Workspace(api.workspace_bytes(Nx, Ns, 1))))
    for (u, Tl, w1) in sub:
        api.loop_step(u, Tl, L, dtau, scheme, 1, ws=w1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for (u, Tl, w1) in sub:
        api.loop_step(u, Tl, L, dtau, scheme, Kp, ws=w1)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t1
    plain = {"value": pts_step * Kp / tp, "unit": "pts/s", "steps": Kp,
             "method": "loop_step per loop, sequential on one stream"}

    cpu = None if args.no_cpu else cpu_baseline(specs, dtau, scheme)
    cpu_all = None if args.no_cpu else cpu_baseline_all_cores(specs, dtau, scheme)
    out = {
        "metric": METRIC,
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": nl, "shapes": [[Nx, Ns]], "L": L, "scheme": cfg["scheme"],
                   "dtau": dtau, "form": "G from the autograd path (LoopCostBand forward + adjoint backward) "
                                         "and the fused update loop_update_grad, band-layout state",
                   "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": gpu_s / steps * 1e3,
        "roofline": roofline, "cpu_baseline": cpu, "cpu_baseline_all_cores": cpu_all,
        "autograd_rfft_layout": {"value": pts_step * k_r / wall_r, "unit": "pts/s", "steps": k_r,
                                 "gpu_ms_per_step": gpu_r / k_r * 1e3,
                                 "method": "LoopCost on rfft-layout tensors + loop_update_grad"},
        "autograd_saved_u": {"value": pts_step * k_r / wall_n, "unit": "pts/s", "steps": k_r,
                             "gpu_ms_per_step": gpu_n / k_r * 1e3,
                             "method": "LoopCostBand with save_u: u on the s grid kept from the forward "
                                       "(k_colR in place of k_colAC), a grid-sized saved tensor"},
        "fused": {"value": pts_step * steps / wall_f, "unit": "pts/s", "steps": steps,
                  "gpu_ms_per_step": gpu_f / steps * 1e3, "schedule": tuning["schedule"],
                  "variants": tuning["variants"], "method": "loop_batch_step (all steps in one call)"},
        "autograd_vs_fused_time": round((gpu_s / steps) / (gpu_f / steps), 3),
        "autograd_vs_fused_max_rel_diff": diff,
        "plain": plain,
        "batched_vs_plain": value / plain["value"],
        "J_mean_end": float(J_end.mean()),
    }
    print(json.dumps(out))


def xi_step_bytes(Nx, Ns):
    """Algorithmic HBM bytes of one centre-symmetric step of one loop: W' = Kx Ns real values
    of one intermediate (8 B), S' = Kx (Ks + 1) complex band values (16 B). B: 2W'; C: 2W' +
    2S'; D: 3W'; E: 2W' + 2S' (reads and writes as in the full step). 8 (9W' + 8S') bytes."""
    Kx, Ks = (Nx - 1) // 3, (Ns - 1) // 3
    W, S = Kx * Ns, Kx * (Ks + 1)
    return 8 * (9 * W + 8 * S)


def bench_xi(args, cfg, specs, steps, dtau, scheme):
    """Centre-symmetric loops through loop_step_xi: the loops of the workload projected onto
    u(-x, s) = -u(x, s), K steps in one call (the conversion in and out of the half state is
    inside the timed region). loop_step on the same projected loops is timed beside it."""
    import numpy as np
    import torch

    from paper_2007_06427_amd import api
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    L = specs[0].L
    Nx, Ns = specs[0].Nx, specs[0].Ns
    nl = len(specs)
    assert all((s.L, s.Nx, s.Ns) == (L, Nx, Ns) for s in specs)
    ws = api.Workspace(api.xi_workspace_bytes(Nx, Ns, nl))
    u0 = torch.from_numpy(np.stack([s.uhat for s in specs])).to(dev)
    T0 = torch.tensor([s.T for s in specs], dtype=torch.float64, device=dev)
    api.loop_step_xi(u0, T0, L, dtau, scheme, 0, ws=ws)  # zero steps: the projection alone

    def timed(fn, k):
        u, T = u0.clone(), T0.clone()
        fn(u, T, args.warmup)
        torch.cuda.synchronize()
        u, T = u0.clone(), T0.clone()
        Jh = torch.zeros(k, nl, dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        fn(u, T, k, Jh)
        e1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3, Jh.cpu().numpy(), u

    wall, gpu_s, J, u = timed(lambda u, T, k, Jh=None: api.loop_step_xi(u, T, L, dtau, scheme, k, J_hist=Jh, ws=ws),
                              steps)
    assert ws.status() == 0 and np.all(np.isfinite(J)), "device flagged a non-finite state"
    wsf = api.Workspace(api.workspace_bytes(Nx, Ns, nl))
    wall_f, gpu_f, J_f, u_f = timed(lambda u, T, k, Jh=None: api.loop_step(u, T, L, dtau, scheme, k, J_hist=Jh,
                                                                           ws=wsf), steps)
    pts = Nx * Ns * nl
    by = xi_step_bytes(Nx, Ns) * nl
    achieved = by * steps / gpu_s / 1e9
    out = {
        "metric": METRIC,
        "value": pts * steps / wall, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": nl, "shapes": [[Nx, Ns]], "scheme": cfg["scheme"],
                   "dtau": dtau, "form": "centre-symmetric (loop_step_xi)", "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": gpu_s / steps * 1e3,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole centre-symmetric step (passes B-E, conversions in and out)",
                     "bytes_per_step": by},
        "cpu_baseline": None,
        "full_path": {"value": pts * steps / wall_f, "unit": "pts/s", "gpu_ms_per_step": gpu_f / steps * 1e3,
                      "method": "loop_step on the same centre-symmetric loops"},
        "xi_vs_full": wall_f / wall,
        "J_rel_diff_vs_full": float(np.max(np.abs(J - J_f) / J_f)),
    }
    print(json.dumps(out))


def expanded_step_bytes(Nx, Ns):
    """Algorithmic HBM bytes of one expanded-form step of one loop (16 B per complex value, W and
    S as in pass_bytes): XB reads A and Cb and writes the transformed G_1NL (3W); XC reads it and
    u_hat and writes u_hat' and the next A and Cb (3W + 2S). 16 (6W + 2S) bytes."""
    W, S = band(Nx, Ns)
    return 16 * (6 * W + 2 * S)


def bench_expanded(args, cfg, specs, steps, dtau, scheme):
    """The paper's expanded form (loop_step_expanded) on the workload's loops, K steps in one call,
    with loop_step on the same loops timed beside it."""
    import numpy as np
    import torch

    from paper_2007_06427_amd import api
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    L = specs[0].L
    Nx, Ns = specs[0].Nx, specs[0].Ns
    nl = len(specs)
    assert all((s.L, s.Nx, s.Ns) == (L, Nx, Ns) for s in specs)
    ws = api.Workspace(api.workspace_bytes(Nx, Ns, nl))
    u0 = torch.from_numpy(np.stack([s.uhat for s in specs])).to(dev)
    T0 = torch.tensor([s.T for s in specs], dtype=torch.float64, device=dev)

    def timed(fn, k):
        u, T = u0.clone(), T0.clone()
        fn(u, T, args.warmup)
        torch.cuda.synchronize()
        u, T = u0.clone(), T0.clone()
        Jh = torch.zeros(k, nl, dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        fn(u, T, k, Jh)
        e1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3, Jh.cpu().numpy()

    wall, gpu_s, J = timed(lambda u, T, k, Jh=None: api.loop_step_expanded(u, T, L, dtau, scheme, k, J_hist=Jh, ws=ws),
                           steps)
    assert ws.status() == 0 and np.all(np.isfinite(J)), "device flagged a non-finite state"
    wall_f, gpu_f, J_f = timed(lambda u, T, k, Jh=None: api.loop_step(u, T, L, dtau, scheme, k, J_hist=Jh, ws=ws),
                               steps)
    pts = Nx * Ns * nl
    by = expanded_step_bytes(Nx, Ns) * nl
    achieved = by * steps / gpu_s / 1e9
    out = {
        "metric": METRIC,
        "value": pts * steps / wall, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": nl, "shapes": [[Nx, Ns]], "scheme": cfg["scheme"],
                   "dtau": dtau, "form": "expanded (eq. KS_G_1, loop_step_expanded)", "parallelism": "none (1 GPU)"},
        "gpu_ms_per_step": gpu_s / steps * 1e3,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole expanded-form step (XB, finalize, XC with the next XA)", "bytes_per_step": by},
        "cpu_baseline": None,
        "full_path": {"value": pts * steps / wall_f, "unit": "pts/s", "gpu_ms_per_step": gpu_f / steps * 1e3,
                      "method": "loop_step on the same loops"},
        "expanded_vs_full": wall_f / wall,
        "J_rel_diff_vs_full": float(np.max(np.abs(J - J_f) / J_f)),
    }
    print(json.dumps(out))


def bench_converge(args, spec, dtau=0.05, J_tol=1e-10, stride=100):
    """The convergence driver (loop_converge) from the loop's seed to J < J_tol, plain and with
    the extrapolations of App. C. `value` is space-time points advanced per second of the
    accelerated run, driver included; the steps saved are reported beside it."""
    import torch

    from paper_2007_06427_amd import api
    dev = "cuda:0"
    runs = {}
    for acc in (False, True):
        u = torch.from_numpy(spec.uhat[None]).to(dev)
        T = torch.tensor([spec.T], dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.loop_converge(u, T, spec.L, dtau, api.IMEX, J_tol, stride=stride, accelerate=acc)
        torch.cuda.synchronize()
        runs[acc] = (r, time.perf_counter() - t0, T.item())
        assert r["steps"][0] > 0, "did not converge"
    (rp, wp, Tp), (ra, wa, Ta) = runs[False], runs[True]
    pts = spec.Nx * spec.Ns
    out = {
        "metric": METRIC,
        "value": pts * ra["steps"][0] / wa, "unit": "pts/s", "n_gpus": 1, "steps": ra["steps"][0], "warmup": 0,
        "ms_per_step": wa / ra["steps"][0] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "loops": 1, "shapes": [[spec.Nx, spec.Ns]], "scheme": "imex",
                   "dtau": dtau, "J_tol": J_tol, "stride": stride, "form": api.step_form(spec.Nx, spec.Ns, 1),
                   "parallelism": "none (1 GPU)"},
        "roofline": None, "cpu_baseline": None,
        "converge": {"plain_steps": rp["steps"][0], "plain_s": round(wp, 3), "accelerated_steps": ra["steps"][0],
                     "accelerated_s": round(wa, 3), "extrapolations": ra["extrapolations"][0],
                     "steps_saved": round(1.0 - ra["steps"][0] / rp["steps"][0], 4),
                     "time_saved": round(1.0 - wa / wp, 4), "J_final": [rp["J"][0], ra["J"][0]],
                     "T_final": [Tp, Ta]},
    }
    print(json.dumps(out))


# periods of the centre-symmetric orbits at L = 39 the paper reports (Sec. 4.4, Fig. 5)
PAPER_PERIODS = [25.37, 53.13, 76.61, 106.98, 123.37, 147.42]


def bench_orbits(args, E=128, per_run=2, chunk=400_000, J_tol=5e-25):
    """Initial loops from chaotic runs (Sec. 4.3) driven to periodic orbits (Sec. 4.4).

    The runs: E centre-symmetric KS runs at L = 39 on 64 modes (ETDRK4, dt = 0.05), started
    from seeded small odd fields, 4000 steps of transient and 20000 recorded steps sampled
    every 2. Pairs of norm maxima within 1% and 20 <= T <= 160 give the loops (the first
    `per_run` pairs of each run; 64 x 64 grid, temporal modes |k| <= 10). loop_converge then
    drives all loops together in chunks of `chunk` steps (IMEX, dtau = 0.15, J examined every
    1000 steps, App. C extrapolations), until J < J_tol (the paper's sqrt(J) < 1e-12 is J < 5e-25
    in the J = 1/2 int int r^2 used here) or --steps steps. `value` is space-time points of
    the loop dynamics advanced per second."""
    import numpy as np
    import torch

    import loopgen
    from paper_2007_06427_amd import api, initial_loops as il
    dev = "cuda:0"
    L, Nx, dt, every = 39.0, 64, 0.05, 2
    total = args.steps if args.steps is not None else 2_000_000
    rng = np.random.default_rng(2020)
    u0 = torch.from_numpy(np.stack([loopgen.random_ks_state(rng, Nx, scale=0.1, odd=True) for _ in range(E)])).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loops, T, triples, norms, snaps = il.initial_loops(u0, L, dt, 4000, 20000, every, 0.01, 20.0, 160.0, Ns=64, kc=10,
                                                       per_run=per_run)
    torch.cuda.synchronize()
    t_pipe = time.perf_counter() - t0
    nl = loops.shape[0]
    T0 = T.cpu().numpy().copy()
    steps = np.full(nl, -1, dtype=np.int64)
    done, t_conv, J = 0, 0.0, None
    while done < total and np.any(steps < 0):
        k = min(chunk, total - done)
        t1 = time.perf_counter()
        r = api.loop_converge(loops, T, L, 0.15, api.IMEX, J_tol, stride=1000, max_steps=k, accelerate=True)
        torch.cuda.synchronize()
        t_conv += time.perf_counter() - t1
        newly = (np.array(r["steps"]) >= 0) & (steps < 0)
        steps[newly] = done + np.array(r["steps"])[newly]
        J = np.array(r["J"])
        done += k
        print(f"# {done} steps: {int(np.sum(steps >= 0))} of {nl} loops below J_tol, "
              f"{int(np.sum(J < 5e-21))} with sqrt(J_paper) < 1e-10", file=sys.stderr, flush=True)
    u = loops.cpu().numpy()
    Tf = T.cpu().numpy()
    # equilibria (no s-dependence) converge with T left free; repeats are multiples of a shorter orbit
    s_energy = np.sum(np.abs(u[:, 1:, :]) ** 2, axis=(1, 2)) / np.maximum(np.sum(np.abs(u) ** 2, axis=(1, 2)), 1e-300)
    found = []
    for i in np.argsort(Tf):
        if J[i] >= 5e-21 or s_energy[i] < 1e-12:
            continue
        if any(abs(Tf[i] - f["T"]) < 1e-3 * f["T"] for f in found):
            next(f for f in found if abs(Tf[i] - f["T"]) < 1e-3 * f["T"])["count"] += 1
            continue
        found.append({"T": round(float(Tf[i]), 4), "sqrtJ_paper": float(np.sqrt(2 * J[i])), "count": 1})
    for f in found:
        base = [g["T"] for g in found if g["T"] < f["T"] and abs(f["T"] / g["T"] - round(f["T"] / g["T"])) < 1e-3]
        f["repeat_of"] = base[0] if base else None
    pts = nl * 64 * 64
    out = {
        "metric": METRIC,
        "value": pts * done / t_conv, "unit": "pts/s", "n_gpus": 1, "steps": done, "warmup": 0,
        "ms_per_step": t_conv / done * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded chaotic KS runs)",
        "config": {"workload": args.workload, "runs": E, "loops": nl, "shapes": [[64, 64]], "L": L, "scheme": "imex",
                   "dtau": 0.15, "J_tol": J_tol, "form": api.step_form(64, 64, nl), "parallelism": "none (1 GPU)"},
        # the loop dynamics run in the resident form: one block per loop, bound by FP64 arithmetic
        # and LDS latency on the CU each loop occupies
        "roofline": {"bound": "alu", "achieved": round(step_flops(64, 64) * nl * done / t_conv / 1e12, 3),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(step_flops(64, 64) * nl * done / t_conv / 1e12 / FP64_PEAK_TFLOPS, 4),
                     "traffic": None, "kernel": "k_resident<64, 64>", "flops_per_step": step_flops(64, 64),
                     "cus_used": min(nl, CUS),
                     "frac_of_cus_used": round(step_flops(64, 64) * nl * done / t_conv / 1e12
                                               / (FP64_PEAK_TFLOPS * min(nl, CUS) / CUS), 4)},
        "cpu_baseline": None,
        "pipeline": {"seconds": round(t_pipe, 3), "run_steps_per_s": E * 24000 / t_pipe,
                     "T0_range": [round(float(T0.min()), 2), round(float(T0.max()), 2)]},
        "orbits": {"converged_below_J_tol": int(np.sum(steps >= 0)),
                   "sqrtJ_paper_below_1e-10": int(np.sum(J < 5e-21)),
                   "equilibria": int(np.sum((J < 5e-21) & (s_energy < 1e-12))),
                   "periods": found,
                   "paper_periods": PAPER_PERIODS,
                   "paper_periods_matched": [p for p in PAPER_PERIODS
                                             if any(abs(f["T"] - p) < 0.01 for f in found)]},
    }
    print(json.dumps(out))


def dns_step_flops(Nx):
    """FP64 flops of one ETDRK4 step of one run (direct transforms, K = (Nx-1)/3 modes): four
    nonlinear evaluations, each an inverse sum over K modes at Nx points and a forward sum over
    Nx points for K + 1 modes (4 flops per complex-by-real term), plus the stage combinations
    (about 40 flops per mode)."""
    K = (Nx - 1) // 3
    return 4 * (4 * Nx * K + 4 * Nx * (K + 1)) + 40 * (K + 1)


def bench_dns(args, E=4096, Nx=64, L=39.0, dt=0.05, every=2):
    """ks_integrate alone: E runs advanced together, norms and states sampled every 2 steps.
    `value` is grid points of the runs advanced per second (Nx per run-step)."""
    import numpy as np
    import torch

    import loopgen
    from paper_2007_06427_amd import api, initial_loops as il
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    steps = args.steps if args.steps is not None else 4000
    steps -= steps % every
    rng = np.random.default_rng(7)
    u = torch.from_numpy(np.stack([loopgen.random_ks_state(rng, Nx, scale=0.1, odd=True) for _ in range(E)])).to(dev)
    il.ks_integrate(u, L, dt, 2000, 2000, True)  # transient, untimed
    ns = steps // every
    norms = torch.empty(E, ns, dtype=torch.float64, device=dev)
    snaps = torch.empty(E, ns, Nx // 2 + 1, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    il.ks_integrate(u, L, dt, steps, every, True, norms, snaps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) * 1e-3
    n = norms.cpu().numpy()
    assert np.all(np.isfinite(n)) and n.min() > 1.0, "runs left the chaotic set"
    fl = dns_step_flops(Nx) * E * steps
    out = {
        "metric": "KS run grid points advanced per second (ETDRK4, FP64)",
        "value": Nx * E * steps / wall, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": 2000,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded chaotic KS runs)",
        "config": {"workload": args.workload, "runs": E, "Nx": Nx, "L": L, "dt": dt, "sample_every": every,
                   "symmetric": True, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "alu", "achieved": round(fl / gpu_s / 1e12, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(fl / gpu_s / 1e12 / FP64_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": f"k_ks_etdrk4<{Nx}>", "flops_per_run_step": dns_step_flops(Nx),
                     "avg_launch_us": round(gpu_s * 1e6, 1),
                     "sample_bytes": int(E * ns * (8 + 16 * (Nx // 2 + 1)))},
        "cpu_baseline": None,
        "norm_range": [float(n.min()), float(n.max())],
    }
    print(json.dumps(out))


def host_cpu() -> str:
    """The host CPU's model name, as /proc/cpuinfo gives it (or 'unknown')."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(specs, dtau, scheme, budget_s=15.0):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same workload: rounds of
    one step of every loop of the workload, in order, until the time budget is spent."""
    pts, dt, rounds = _oracle_rounds([(s.L, s.Nx, s.Ns, s.T, s.uhat) for s in specs], dtau, scheme, budget_s)
    return {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle", "cpu": host_cpu(),
            "sample": f"{pts} space-time points in {dt:.1f} s: {rounds} round(s) of one step of each of the "
                      f"{len(specs)} loops, in order (NumPy FP64, one process, one thread)"}


def _oracle_rounds(loops, dtau, scheme, budget_s):
    """One oracle step of each loop in turn, round after round, until budget_s has passed.
    Returns (space-time points stepped, seconds, rounds begun)."""
    from oracle import ks_loop as K
    state = [[u, T] for (_, _, _, T, u) in loops]
    t0 = time.perf_counter()
    pts, rounds = 0, 0
    while loops and time.perf_counter() - t0 < budget_s:
        rounds += 1
        for (L, Nx, Ns, _, _), st in zip(loops, state):
            if time.perf_counter() - t0 >= budget_s:
                break
            st[0], st[1], _ = K.step(st[0], st[1], L, dtau, scheme, 1)
            pts += Nx * Ns
    return pts, time.perf_counter() - t0, rounds


def _oracle_worker(job):
    """_oracle_rounds on a share of the loops (a spawned process: no GPU, NumPy only)."""
    loops, dtau, scheme, budget_s = job
    return _oracle_rounds(loops, dtau, scheme, budget_s)[0]


def cpu_baseline_all_cores(specs, dtau, scheme, budget_s=15.0, cores=None):
    """The same oracle in one spawned process per host core (up to 16, the host share of one
    GPU), each taking rounds over every cores-th loop of the workload within the budget."""
    import multiprocessing as mp
    cores = cores or min(16, os.cpu_count() or 1)
    jobs = [([(s.L, s.Nx, s.Ns, s.T, s.uhat) for s in specs[c::cores]], dtau, scheme, budget_s)
            for c in range(cores)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_worker, [([], dtau, scheme, 0.0)] * cores)  # interpreters started and NumPy imported
        t0 = time.perf_counter()
        pts = sum(pool.map(_oracle_worker, jobs))
        dt = time.perf_counter() - t0
    return {"value": pts / dt, "unit": "pts/s", "cores": cores, "kind": "oracle", "cpu": host_cpu(),
            "sample": f"{pts} space-time points in {dt:.1f} s: rounds of one step of each loop, the loops "
                      f"dealt over {cores} processes (NumPy FP64, one thread each)"}


if __name__ == "__main__":
    main()
