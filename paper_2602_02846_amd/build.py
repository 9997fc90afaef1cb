"""Builds the planner library libkpx.so for gfx950 with hipcc (in-tree)."""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "kpx.hip")
SRC_DIFF = os.path.join(HERE, "csrc", "kpx_diff.hip")
DEPS = [SRC, SRC_DIFF, os.path.join(HERE, "csrc", "kpx_device.hpp"),
        os.path.join(HERE, "csrc", "kpx_diff_device.hpp"),
        os.path.join(os.path.dirname(HERE), "include", "kpx.h")]
LIB = os.path.join(HERE, "libkpx.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # packed float32 instructions stay off (the compiler would otherwise form them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the planner library cannot be built")
    return exe


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile libkpx.so.  With force=False an up-to-date library is kept."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(p) for p in DEPS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-o", tmp, SRC, SRC_DIFF]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
