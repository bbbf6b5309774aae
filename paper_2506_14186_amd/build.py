"""Build libdmx.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmx.so")
# translation units, compiled in parallel and linked into one library: the
# host side (C ABI, dispatch, tapes, server) and one unit per kernel family
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("dmx_lib.hip", "kern_free_small.hip", "kern_free.hip",
                                                    "kern_free_wide.hip", "kern_tree.hip", "kern_stack.hip")]
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are not generated
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


KERNEL_SOURCES = ["dmx_common.hpp", "dmx_free.hpp", "dmx_tree.hpp", "dmx_rk.hpp", "dmx_geom.hpp", "dmx_stack.hpp",
                  "dmx_stack_rk.hpp", "dmx_stack_adj.hpp"]


def kernel_digest():
    """sha256 of the device-code headers (the forward/reverse kernels), used to
    tell whether recorded hardware counters still describe the built kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def build(verbose=False, extra=()):
    """Compile every translation unit (in parallel) and link libdmx.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + list(extra) + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc " + " ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
