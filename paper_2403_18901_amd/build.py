"""Builds the HIP library libgdg_hip.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgdg_hip.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("gdg_kernels.hip", "gdg_mlp.hip", "gdg_host.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # keep the compiler from emitting packed-FP32 (v_pk_*_f32) instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


# the LDS bandwidth probe behind the decode kernel's roofline peak (its own library)
PROBE_LIB = os.path.join(HERE, "libgdg_probe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "lds_probe.hip")]


def _hipcc(sources, out, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC] + FLAGS + sources + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _hipcc(SOURCES, LIB, verbose)
    _hipcc(PROBE_SOURCES, PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
