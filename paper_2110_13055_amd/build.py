"""Build libcdi.so (HIP, gfx950) in-tree.

    python -m paper_2110_13055_amd.build

Compiles the seeded primitive generator (C) with gcc and every HIP source of
``csrc/`` with hipcc for gfx950 into ``paper_2110_13055_amd/libcdi.so``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcdi.so")
ARCH = os.environ.get("CDI_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b+c only inside one source expression, so a device function
    # rounds identically in every kernel it is inlined into (a batched step
    # must reproduce the single-instance step bit for bit)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd, quiet=False):
    if not quiet:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the GPU-only feature flag; drop that note
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if err.strip():
        print(err, file=sys.stderr, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def build(verbose: bool = True) -> str:
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    gen_o = os.path.join(bdir, "geomgen.o")
    # the generator's porosity stop rule is floating point: the same source,
    # compiler and flags as the CPU reference's copy, no contraction
    _run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-c", os.path.join(HERE, "inputs", "geomgen.c"),
          "-o", gen_o])
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    incs = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            "-I", os.path.join(HERE, "inputs")]
    objs = []
    procs = []
    for src in srcs:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = ["hipcc", *HIP_FLAGS, *incs, "-c", src, "-o", obj]
        print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
    for cmd, p in procs:
        _, err = p.communicate()
        err = "\n".join(l for l in err.splitlines()
                        if "is not a recognized feature for this target" not in l)
        if err.strip():
            print(err, file=sys.stderr, flush=True)
        if p.returncode != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, gen_o, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
