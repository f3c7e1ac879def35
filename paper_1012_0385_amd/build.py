"""Build of the gfx950 shared library ``libasep.so`` (in-tree, with hipcc)."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libasep.so")
SOURCES = ["asep_kernels.hip", "asep_sweep_plain.hip", "asep_sweep_disorder.hip",
           "asep_sweep_two_lane.hip", "asep_host.cpp", "asep_server.cpp", "asep_server_hip.cpp", "asep_noalloc.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _flags():
    return [
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        # packed FP32 forms are kept out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-Wall",
        "-Wno-unused-function",
    ]


HEADERS = [os.path.join(CSRC, h) for h in ("asep_device.h", "asep_internal.h", "asep_serve.h")] + [
    os.path.join(ROOT, "include", "asep.h")]


def _stale(path: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [path] + HEADERS if os.path.exists(f))


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source of the library and link libasep.so.  By default
    everything is recompiled; with incremental=True only objects older than
    their source or a shared header are."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        if incremental and not _stale(path, obj):
            objs.append(obj)
            continue
        cmd = [cc] + _flags() + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n%s\n%s" % (" ".join(cmd), out.decode(errors="replace")))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys

    print(build(verbose=True, incremental="--incremental" in sys.argv))
