"""Compile the HIP library liblooporbit.so for gfx950, in-tree, with hipcc.

Usage: python -m paper_2007_06427_amd.build   (or call build()).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("looporbit.hip", "ksdns.hip")]
OUT = os.path.join(HERE, "liblooporbit.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are disabled on this target (they are not used by FP64 code anyway)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-value", "-Wno-unused-result",
    # every product and sum rounded on its own (no fused multiply-add contraction): the same
    # expression then gives the same bits in every kernel that inlines it, whatever the
    # surrounding code, so the batched, resident and per-pass forms agree bit for bit
    "-ffp-contract=off",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs = [OUT + "." + os.path.splitext(os.path.basename(s))[0] + ".o" for s in SRCS]
    procs = [subprocess.Popen([hipcc(), *FLAGS, *inc, "-c", s, "-o", o], stdout=subprocess.PIPE,
                              stderr=subprocess.PIPE, text=True) for s, o in zip(SRCS, objs)]
    failed = False
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed = True
        elif verbose:
            sys.stderr.write(err)
    if failed:
        raise RuntimeError("hipcc failed building liblooporbit.so")
    tmp = OUT + ".tmp"
    res = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                         capture_output=True, text=True)
    for o in objs:
        os.remove(o)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking liblooporbit.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
