"""Compile the HIP library libhpsleaf.so for gfx950, in place.

Run as ``python -m paper_2211_14969_amd.build``.  Every source under csrc/ is
compiled into one shared object next to this file; the test suite's
instruction probe (tests/probe) is compiled beside its source.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhpsleaf.so")
ARCH = "gfx950"

SOURCES = ["hps_kernels.hip", "hps_abi.hip", "hps_iface.hip", "hps_cheb.cpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# The instruction probe of the test suite (tests/probe), built beside it.
PROBE_SRC = os.path.join(HERE, "..", "tests", "probe", "mfma_probe.hip")
PROBE_LIB = os.path.join(HERE, "..", "tests", "probe", "libmfmaprobe.so")


def _compile(srcs, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(HERE, "..", "include"),
           *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _compile([os.path.join(CSRC, s) for s in SOURCES], LIB, verbose)
    if os.path.exists(PROBE_SRC):
        _compile([PROBE_SRC], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
