"""Build the gfx950 shared library ``libbemc.so`` in the package directory.

hipcc compiles the kernels for gfx950 (cross-compiles without a GPU) as code-object
version 5, which every ROCm 7 runtime loads (the process may run on torch's bundled HIP
runtime, see bemc.load_library).  Packed FP32
instructions are disabled for every HIP source (``-packed-fp32-ops``); FP64 atomic adds
use the hardware instruction (``-munsafe-fp-atomics``, device memory is coarse-grained).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbemc.so")
SOURCES = ["kernels.hip", "order.hip", "near_order.hip", "noalloc.hip", "api.cpp", "server.cpp", "solver.cpp", "rules.cpp"]
# measurement only (issue rates of the far kernels' instruction classes, read by the benchmark)
PROBE_LIB = os.path.join(HERE, "libissue_probe.so")
PROBE_SOURCE = "issue_probe.hip"
ARCH = os.environ.get("BEMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
              "-I", INCLUDE, "-I", CSRC,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
              "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + lang + common + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
        if msgs.strip() and verbose:
            print(msgs)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-fPIC", "-o", tmp] + objs + [
        "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    # the issue-rate probe: a library of its own, so that the evaluation path does not carry it
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc(), "-x", "hip"] + common + ["-shared", "-o", tmp, os.path.join(CSRC, PROBE_SOURCE)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"hipcc failed on {PROBE_SOURCE}:\n{msgs}")
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
