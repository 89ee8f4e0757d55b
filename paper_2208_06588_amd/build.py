"""Build the in-tree HIP library ``libalew.so`` for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("alew.hip", "alew2d.hip")]
DEPS = [os.path.join(HERE, "csrc", f)
        for f in ("alew.hip", "alew2d.hip", "alew_device.h", "alew_kernels.h", "alew_adjoint.h")]
LIB = os.path.join(HERE, "libalew.so")
INCLUDE = os.path.join(ROOT, "include")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # multiply-adds fused only within one source expression, so a tile body
    # rounds the same way wherever it is inlined (engines agree bit for bit)
    "-ffp-contract=on",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile csrc/alew.hip and csrc/alew2d.hip into libalew.so (always, unless force=False and
    the library is newer than every source)."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(d) <= t for d in DEPS + [os.path.join(INCLUDE, "alew.h")]):
            return LIB
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", INCLUDE, "-o", tmp, *SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
