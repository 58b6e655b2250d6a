"""Summaries of rocprofv3 output for profiles/: per-kernel durations and HBM traffic.

    python -m paper_2007_06427_amd.profiling trace <kernel_stats.csv> <out.md> <workload> "<command>"
    python -m paper_2007_06427_amd.profiling traffic <fetch.csv> <write.csv> <workload> "<command>"

`traffic` reads two counter-collection runs of the same command: FETCH_SIZE in one and
WRITE_SIZE in the other, both in KiB per dispatch. It scales each counter by its reading for a
plain device copy of known size. bench.py runs a 64 MiB device copy for this, so a
calibrated counter reads 65536 KiB for that copy. It then writes
profiles/traffic_<workload>.{json,md}, stamped with a digest of the sources of the workload's translation unit (the file and the
project headers it includes); bench.py uses the bytes only while those are unchanged.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 64 << 20


def _unit_files(unit: str):
    """The translation unit csrc/<unit> and every kernel header (csrc/) it includes, recursively.
    The C-ABI headers under include/ hold declarations only and are left out."""
    dirs = [os.path.join(HERE, "csrc")]
    seen, todo = [], [os.path.join(HERE, "csrc", unit)]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.append(f)
        for inc in re.findall(r'^#include "([^"]+)"', open(f).read(), flags=re.M):
            for d in dirs:
                if os.path.exists(os.path.join(d, inc)):
                    todo.append(os.path.join(d, inc))
                    break
    return sorted(seen)


def source_digest(unit: str = "looporbit.hip") -> str:
    """Digest of the sources that make one translation unit's kernels (the loop dynamics by
    default; ksdns.hip for the initial-loop pipeline)."""
    h = hashlib.sha256()
    for f in _unit_files(unit):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def unit_of(workload: str) -> str:
    return "ksdns.hip" if workload.startswith("ks-dns") else "looporbit.hip"


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name).strip()


def summarize_trace(stats_csv: str, out_md: str, workload: str, command: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel durations: {workload}", "",
             f"Command (run from the repository root, with `TMPDIR=/tmp`): `{command}`", "",
             f"Kernel source digest: `{source_digest(unit_of(workload))}`", "",
             "| kernel | calls | avg us | total ms | % of GPU time |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    trace_csv = stats_csv.replace("kernel_stats", "kernel_trace")
    if trace_csv != stats_csv and os.path.exists(trace_csv):
        lines += _per_grid(trace_csv, [short_name(r["Name"]) for r in rows if short_name(r["Name"]).startswith("k_")])
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_grid(trace_csv: str, kernels) -> list:
    """Launch durations of the given kernels, split by grid size: a kernel launched over all
    loops, over groups of them (the streams schedule) or over one loop (the plain method) has one
    row per grid, so that the launches over all loops can be read apart."""
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        k = short_name(r["Kernel_Name"])
        if k in kernels:
            acc[(k, int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y", 1) or 1))].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["", "Per grid size (work-items), from the kernel trace of the same run:", "",
             "| kernel | grid | launches | avg us | min us | max us |", "|---|---:|---:|---:|---:|---:|"]
    for (k, g), v in sorted(acc.items(), key=lambda kv: (kernels.index(kv[0][0]), -kv[0][1])):
        lines.append(f"| `{k}` | {g} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    return lines


def _per_kernel(counter_csv: str, counter: str):
    acc = collections.defaultdict(list)
    grids = {}
    for r in csv.DictReader(open(counter_csv)):
        if r["Counter_Name"] != counter:
            continue
        k = short_name(r["Kernel_Name"])
        acc[(k, r["Grid_Size"])].append(float(r["Counter_Value"]))
        grids[(k, r["Grid_Size"])] = int(r["Grid_Size"])
    return acc


def _calibration_copy(counter_csv: str, counter: str):
    """The reading of the first copy dispatch among those with the largest grid of the run.

    The device copy kernel's grid stops growing at a few megabytes, so copies of 64 MiB and
    larger share one grid; bench.py makes its 64 MiB copy before any other large copy."""
    rows = [r for r in csv.DictReader(open(counter_csv))
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
    if not rows:
        return None
    big = max(int(r["Grid_Size"]) for r in rows)
    first = min((r for r in rows if int(r["Grid_Size"]) == big), key=lambda r: int(r["Dispatch_Id"]))
    return float(first["Counter_Value"])


def summarize_traffic(fetch_csv: str, write_csv: str, workload: str, command: str) -> None:
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    # calibration: bench.py makes the known 64 MiB copy before any other copy of the run
    want_kib = COPY_BYTES / 1024
    fcopy, wcopy = _calibration_copy(fetch_csv, "FETCH_SIZE"), _calibration_copy(write_csv, "WRITE_SIZE")
    ffac = (fcopy / want_kib) if fcopy else 1.0
    wfac = (wcopy / want_kib) if wcopy else 1.0
    # Per kernel, the launch over every loop of the plan (the largest grid), taken from
    # dispatches of the same grid in both runs: a schedule that splits the loops into groups
    # also launches the kernel on part of them, and the two runs may tune differently.
    kernels = {}
    for key in sorted(set(fetch) & set(write), key=lambda k: (k[0], -int(k[1]))):
        name = key[0]
        if not name.startswith("k_"):
            continue
        if name in kernels:
            continue
        f = sum(fetch[key]) / len(fetch[key])
        w = sum(write[key]) / len(write[key])
        b = (f / ffac + w / wfac) * 1024
        kernels[name] = {"grid": int(key[1]), "fetch_kib": round(f, 1), "write_kib": round(w, 1),
                         "bytes_per_launch": round(b), "dispatches": min(len(fetch[key]), len(write[key]))}
    out = {"workload": workload, "command": command, "source_digest": source_digest(unit_of(workload)),
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": fcopy, "write_kib": wcopy,
                                "fetch_factor": ffac, "write_factor": wfac},
           "kernels": kernels}
    pj = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    json.dump(out, open(pj, "w"), indent=1)
    lines = [f"# HBM traffic per dispatch: {workload}", "",
             f"Two counter runs of: `{command}` with `--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`.", "",
             f"Calibration: a {COPY_BYTES >> 20} MiB device copy read FETCH_SIZE {fcopy} KiB and WRITE_SIZE {wcopy} KiB "
             f"(factors {ffac:.3f}, {wfac:.3f}); kernel readings are divided by these.", "",
             f"Kernel source digest: `{source_digest(unit_of(workload))}`", "",
             "Per kernel: the launches over every loop (largest grid) found in both runs.", "",
             "| kernel | grid (work-items) | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated bytes / launch |",
             "|---|---:|---:|---:|---:|---:|"]
    for k, v in kernels.items():
        lines.append(f"| `{k}` | {v['grid']} | {v['dispatches']} | {v['fetch_kib']} | {v['write_kib']} | "
                     f"{v['bytes_per_launch']} |")
    open(os.path.join(ROOT, "profiles", f"traffic_{workload}.md"), "w").write("\n".join(lines) + "\n")


def summarize_counters(p1_csv: str, p2_csv: str, workload: str, command: str) -> None:
    """SQ counters of the per-pass kernels from two --pmc runs (wave-cycle fractions from the
    first, instruction counts and LDS bank-conflict cycles from the second), per kernel at its
    largest grid, averaged over dispatches."""
    def load(path):
        acc = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(path)):
            acc[(short_name(r["Kernel_Name"]), int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}
    a, b = load(p1_csv), load(p2_csv)
    best = {}
    for (k, g) in set(a) & set(b):
        if k.startswith("k_") and (k not in best or g > best[k]):
            best[k] = g
    lines = [f"# SQ counters per dispatch: {workload}", "",
             f"Two counter runs of: `{command}`, the first with `--pmc SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
             "SQ_WAIT_INST_LDS SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM "
             "SQ_WAVES`, the second with `--pmc SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_LDS_ADDR_CONFLICT "
             "SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INST_LEVEL_LDS SQ_LDS_UNALIGNED_STALL`.", "",
             f"Kernel source digest: `{source_digest(unit_of(workload))}`", "",
             "Fractions are of SQ_WAVE_CYCLES. Conflict cycles are summed over the chip.", "",
             "| kernel | grid | waves | VALU active | LDS active | waiting (any) | waiting (LDS) | LDS insts | "
             "VALU insts | LDS conflict cycles | conflict cycles / LDS inst |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(best):
        A, B = a[(k, best[k])], b[(k, best[k])]
        wc = max(A.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        li = B.get("SQ_INSTS_LDS", 0.0)
        lines.append(f"| `{k}` | {best[k]} | {A.get('SQ_WAVES', 0):.0f} | {A.get('SQ_ACTIVE_INST_VALU', 0) / wc:.2f} | "
                     f"{A.get('SQ_ACTIVE_INST_LDS', 0) / wc:.2f} | {A.get('SQ_WAIT_INST_ANY', 0) / wc:.2f} | "
                     f"{A.get('SQ_WAIT_INST_LDS', 0) / wc:.2f} | {li:.3g} | {B.get('SQ_INSTS_VALU', 0):.3g} | "
                     f"{B.get('SQ_LDS_BANK_CONFLICT', 0):.3g} | {B.get('SQ_LDS_BANK_CONFLICT', 0) / max(li, 1):.1f} |")
    open(os.path.join(ROOT, "profiles", f"counters_{workload}.md"), "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "counters":
        summarize_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    elif sys.argv[1] == "trace":
        summarize_trace(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    elif sys.argv[1] == "traffic":
        summarize_traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        raise SystemExit(__doc__)
