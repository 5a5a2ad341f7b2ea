"""Build the stls shared library for gfx950 in-tree (hipcc, no JIT cache).

    python paper_1809_10026_amd/build.py

The library lands next to this file as ``libstls.so``; the Python binding
loads it from there.  Always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstls.so")
SOURCES = ["stls_host.cpp", "stls_geometry.cpp", "stls_kernels.hip", "stls_fd.hip", "stls_diff.hip", "stls_batch.hip",
           "stls_norms.hip", "stls_mapped.hip"]

# Packed FP32 instructions are kept off on purpose: the compiler would emit
# them from ordinary float code otherwise.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the stls library needs ROCm's hipcc")
    return exe


def batch_source_hash() -> str:
    """SHA-256 of the batched kernels' sources: the key under which the
    batch autotuner caches its choices (a changed kernel is re-tuned)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("stls_batch.hip", "stls_buf.h", "stls_internal.h"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    """Compile every translation unit in parallel, then link libstls.so."""
    tmp = LIB + ".tmp"
    jobs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        defs = [f'-DSTLS_BATCH_SOURCE_HASH="{batch_source_hash()}"'] if src == "stls_batch.hip" else []
        cmd = [hipcc(), *HIP_FLAGS, *lang, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    objs = []
    failed = []
    for src, obj, proc in jobs:
        _, err = proc.communicate()
        errs = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if proc.returncode != 0:
            failed.append(f"compiling {src} failed:\n{errs}")
        elif verbose and errs:
            print(errs)
        objs.append(obj)
    if failed:
        raise RuntimeError("\n".join(failed))
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("linking libstls.so failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    build_mem_patterns()
    return LIB


def build_mem_patterns() -> str:
    """The memory-pattern reference executable (access orders of the hot
    kernels without their arithmetic; see mem_patterns.hip)."""
    exe = os.path.join(HERE, "mem_patterns")
    cmd = [hipcc(), *HIP_FLAGS, "-x", "hip", os.path.join(HERE, "mem_patterns.hip"), "-o", exe + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building mem_patterns failed:\n" + r.stderr)
    os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
