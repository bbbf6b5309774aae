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
                                                    "kern_free_wide.hip", "kern_tree.hip", "kern_stack.hip",
                                                    "kern_stack_params.hip")]
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are not generated
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


DIGEST = os.path.join(HERE, "kern_stack.digest")
LLVM = os.environ.get("ROCM_LLVM", "/opt/rocm/llvm/bin")


def machine_code_digest(obj):
    """sha256 prefix of the gfx950 machine code (.text of the device code
    object) built into a HIP object file: unchanged by edits that leave the
    kernels' instructions as they were."""
    import hashlib
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        fat, co, text = (os.path.join(d, n) for n in ("fat.bin", "dev.co", "text.bin"))
        subprocess.check_call(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", obj, fat])
        subprocess.check_call([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                               f"--input={fat}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"])
        subprocess.check_call([os.path.join(LLVM, "llvm-objcopy"), "-O", "binary", "--only-section=.text", co, text])
        with open(text, "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_digest():
    """Digest of the built cube-stack kernels' machine code (written by build()
    next to the library), used to tell whether recorded hardware counters still
    describe the built kernels; None if the library was built without it."""
    try:
        with open(DIGEST) as f:
            return f.read().strip() or None
    except OSError:
        return None


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
    with open(DIGEST, "w") as f:
        f.write(machine_code_digest(os.path.join(OBJ_DIR, "kern_stack.hip.o")) + "\n")
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
