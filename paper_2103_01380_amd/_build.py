"""Build ``libspid.so`` for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "spid.hip")
OUT = os.path.join(HERE, "libspid.so")
# stand-alone attainable-rate probe (MFMA, HBM, sketch-matrix generation)
PROBE_SRC = os.path.join(HERE, "csrc", "rate_probe.hip")
PROBE_OUT = os.path.join(HERE, "rate_probe")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # keep hipcc from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(flags, src, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc(), *flags, src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-8000:])
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _compile(FLAGS, SRC, OUT, verbose)
    exe_flags = [f for f in FLAGS if f not in ("-shared", "-fPIC")]
    _compile(exe_flags, PROBE_SRC, PROBE_OUT, verbose)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
