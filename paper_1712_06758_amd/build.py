"""Build the gfx950 shared library ``_lib/libspde.so`` with hipcc.

Usage: python -m paper_1712_06758_amd.build   (or call build()).
The library is always rebuilt; hipcc cross-compiles without a GPU present.
The translation units compile in parallel, then link into one library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib", "libspde.so")
OBJ = os.path.join(HERE, "_lib", "obj")
ARCH = os.environ.get("SPDE_OFFLOAD_ARCH", "gfx950")

# the multigrid kernels of each level precision and the operator pass are
# translation units of their own, so that they compile side by side
SOURCES = ["spde_kernels.hip", "spde_operator.hip", "spde_mg_f32.hip", "spde_mg_f64.hip", "spde.cpp",
           "transfer_build.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # no packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the register-pressure trackers of the AMDGPU scheduler: the float fine
    # up-kernels spill 8 instead of 16 B per lane and run 3 % faster
    "-mllvm", "-amdgpu-use-amdgpu-trackers=1",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    procs = []
    objs = []
    for s in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        cmd = [hipcc] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = []
    for s, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed.append(s)
    if failed:
        raise RuntimeError(f"hipcc failed compiling {', '.join(failed)}")
    tmp = OUT + ".tmp"
    cmd = [hipcc] + FLAGS + ["-shared"] + objs + ["-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libspde.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
