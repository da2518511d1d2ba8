"""Build ``libnefty_heat.so`` for gfx950 with hipcc, in-tree.

``python -m paper_2603_11045_amd.build`` compiles the HIP sources under
``csrc/`` into ``paper_2603_11045_amd/libnefty_heat.so`` (the library the
Python binding loads). Every HIP translation unit is compiled with packed
FP32 instructions disabled; the translation units compile in parallel and are
linked against the roctx range library (host-side profiler ranges).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnefty_heat.so")
SOURCES = ["nh_api.hip", "nh_serve.hip", "nh_policy.cpp"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
LINK_LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    """Compile the library (always) and return its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="nh_build_") as objdir:
        procs, objs = [], []
        for s in SOURCES:
            obj = os.path.join(objdir, s + ".o")
            cmd = [hipcc, *[f for f in HIPCC_FLAGS if f != "-shared"], f"-I{INCLUDE}", f"-I{CSRC}", "-c", "-o", obj,
                   os.path.join(CSRC, s)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
            objs.append(obj)
        failed = False
        for p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                sys.stderr.write(out)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed to compile libnefty_heat.so's sources")
        cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *objs, *LINK_LIBS]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed to link libnefty_heat.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
