"""Build libnep.so in-tree with hipcc for gfx950.

    python -m paper_2507_00528_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libnep.so")
SOURCES = [os.path.join(HERE, "csrc", "nep_lib.hip")]
HEADERS = [os.path.join(HERE, "csrc", "nep_device.h"), os.path.join(HERE, "csrc", "nep_kernels.h"),
           os.path.join(HERE, "csrc", "nep_highl.h"),
           os.path.join(ROOT, "include", "nep.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=fast",
    # packed FP32 (v_pk_*_f32) stays off for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = True, extra=None) -> str:
    cmd = [HIPCC, *FLAGS, *(extra or []), "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnep.so")
    noise = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                      if "packed-fp32-ops" not in l and l.strip())
    if verbose and noise:
        print(noise)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
