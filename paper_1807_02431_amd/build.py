"""Builds libgpr_hip.so (gfx950) in place with hipcc, and its timer build libgpr_hip_probe.so
(the same sources with GPR_PHASE_PROBE: the persistent kernel's phase timers, for measurement)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpr_hip.so")
PROBE_LIB = os.path.join(HERE, "libgpr_hip_probe.so")
SOURCES = ["gpr_kernels.hip", "gpr_api.hip"]
HEADERS = ["gpr_device.h", "gpr_kernels.h"]
ARCH = os.environ.get("GPR_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no FMA contraction: the plain and persistent paths must round identically
    "-ffp-contract=off",
    # packed FP32 VALU forms are disabled on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, probe: bool = False) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    bdir = os.path.join(HERE, "_build", "probe" if probe else "lib")
    os.makedirs(bdir, exist_ok=True)
    lib = PROBE_LIB if probe else LIB
    objs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc] + FLAGS + (["-DGPR_PHASE_PROBE"] if probe else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, cwd=bdir, stderr=subprocess.PIPE if not verbose else None)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp], check=True, cwd=bdir)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, probe="--probe" in sys.argv))
