"""Build step of libxdrop.so (hipcc, gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "xdrop_kernels.hip"), os.path.join(HERE, "csrc", "seed_kernels.hip"),
           os.path.join(HERE, "csrc", "xdrop_capi.cpp")]
LIB = os.path.join(HERE, "libxdrop.so")
# measuring tool (int32 VALU peak of the GPU), loaded only by bench.py
PROBE_SOURCES = [os.path.join(HERE, "csrc", "valu_probe.hip")]
PROBE_LIB = os.path.join(HERE, "libxdrop_probe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed-FP32 instructions disabled for all device code; the host pass of
# hipcc prints a harmless "not a recognized feature" note for it.
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_library(out: str = LIB, extra=None, verbose: bool = False, sources=None) -> str:
    cmd = [HIPCC] + FLAGS + (extra or [])
    for src in (sources or SOURCES):
        cmd += ["-x", "hip", src]
    cmd += ["-o", out + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(out + ".tmp", out)
    return out


def build_probe(verbose: bool = False) -> str:
    return build_library(PROBE_LIB, verbose=verbose, sources=PROBE_SOURCES)


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
    print(build_probe(verbose="-v" in sys.argv))
