"""Compile the HIP library (librayshoot.so) for gfx950 in-tree.

Flags that matter for correctness:
  -ffp-contract=off   no implicit FMA anywhere; the deflection loop asks for
                      fused multiply-adds explicitly, and the FP64 re-check
                      keeps the definition's separate multiply and add;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions (the host pass warns that it
                      does not know the feature; that warning is harmless).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librayshoot.so")
ARCH = os.environ.get("RAYSHOOT_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-shared", "-std=c++17",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable", "-Wno-pass-failed",
         f"-I{INCLUDE}", f"-I{CSRC}", "-lpthread"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source into librayshoot.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    proc = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in proc.stderr.splitlines() if noise not in l)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


def asm(out_path: str) -> str:
    """Device assembly of every HIP source (for inspection of the gfx950 code)."""
    parts = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-lpthread")], "--cuda-device-only", "-S",
               src, "-o", "-"]
        proc = subprocess.run(cmd, capture_output=True, text=True, check=True)
        parts.append(proc.stdout)
    with open(out_path, "w") as f:
        f.write("\n".join(parts))
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
