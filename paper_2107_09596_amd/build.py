"""Build libatmgrit.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libatmgrit.so")
SOURCES = ["atm_kernels.hip", "atm_mixed.hip", "atm_large.hip", "atm_pair.hip", "atm_batch.hip", "atm_cnn.hip", "atm_cnn_api.hip", "atm_api.hip"]
HEADERS = ["atm_device.hpp", "atm_kernels.hpp"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one source expression, so that every instantiation of a
    # body (exact or masked tiling, alone or batched) rounds the same way
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every source (always, in parallel), link, and atomically replace the library."""
    compile_flags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="atm_build_") as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = ["hipcc", *compile_flags, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd))
            procs.append((cmd, subprocess.Popen(cmd, cwd=CSRC)))
            objs.append(obj)
        for cmd, proc in procs:
            if proc.wait() != 0:
                raise subprocess.CalledProcessError(proc.returncode, cmd)
        tmp = LIB + ".tmp"
        cmd = ["hipcc", "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
