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
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librayshoot.so")
OBJ_DIR = os.path.join(ROOT, "_build", "rayshoot")
ARCH = os.environ.get("RAYSHOOT_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMPILE_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
                 "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable", "-Wno-pass-failed",
                 f"-I{INCLUDE}", f"-I{CSRC}"]
LINK_FLAGS = [f"--offload-arch={ARCH}", "-fPIC", "-shared", "-lpthread", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
FLAGS = COMPILE_FLAGS + ["-shared", "-lpthread"]
NOISE = "is not a recognized feature for this target"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd))
    proc = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in proc.stderr.splitlines() if NOISE not in l)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}): {' '.join(cmd)}\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP/C++ source (one hipcc per file, in parallel) and link
    librayshoot.so. Always rebuilds every object."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJ_DIR, os.path.basename(s) + ".o") for s in srcs]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _run([HIPCC, *COMPILE_FLAGS, "-c", so[0], "-o", so[1]], verbose),
                    zip(srcs, objs)))
    tmp = LIB + ".tmp"
    _run([HIPCC, *LINK_FLAGS, *objs, "-o", tmp], verbose)
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
