"""Build libdrf.so (host C++ + gfx950 HIP kernels) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdrf.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# packed fp32 instructions stay off in all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), err))
    return err


def build(verbose: bool = False) -> str:
    """Compile every source and link libdrf.so; always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, is_hip in (("host.cpp", False), ("babycuda.cpp", False), ("api.cpp", False), ("kernels.hip", True)):
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + COMMON + ["--offload-arch=" + ARCH] + DEVICE_FLAGS
        cmd += (["-x", "hip"] if is_hip else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        msg = _run(cmd)
        if verbose and msg:
            print(msg, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
