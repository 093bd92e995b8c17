"""Build liblbmhpde.so (HIP kernels for gfx950 + host runtime) in-tree.

    python -m paper_0907_1720_amd.build

Every call recompiles.  Device code is compiled with packed-FP32 instructions
disabled and without floating-point contraction beyond the explicit fused
multiply-adds written in the kernels.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbmhpde.so")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
ARCH = "gfx950"

DEVICE_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-ffp-contract=off",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include", "-Wall", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build step failed: " + " ".join(cmd) + "\n" + out)
    return out


LATTICES = (4, 5, 6, 7)


def build(verbose: bool = False) -> str:
    """Compiles the host sources, the read-out/launcher unit, the boundary-wave
    unit and one kernel unit per lattice size (kernels_q.hip with LBM_Q = 4..7)
    in parallel, then links."""
    os.makedirs(BUILD, exist_ok=True)
    inc = [f"-I{INCLUDE}", f"-I{CSRC}"]
    steps = []
    for src in ("coeffs.cpp", "runtime.cpp"):
        obj = os.path.join(BUILD, src + ".o")
        steps.append((obj, [CLANG] + HOST_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj]))
    for src in ("kernels.hip", "kernels_wave.hip", "noalloc.hip"):
        obj = os.path.join(BUILD, src + ".o")
        steps.append((obj, [HIPCC] + DEVICE_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj]))
    for q in LATTICES:
        obj = os.path.join(BUILD, f"kernels_q{q}.hip.o")
        steps.append((obj, [HIPCC] + DEVICE_FLAGS + inc + [f"-DLBM_Q={q}", "-c",
                                                            os.path.join(CSRC, "kernels_q.hip"), "-o", obj]))
    # the D1Q7 and D1Q5 units take longest: start them first
    steps.sort(key=lambda st: ("q7" not in st[0], "q5" not in st[0]))
    jobs = max(1, min(len(steps), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as pool:
        list(pool.map(lambda st: _run(st[1]), steps))
    objs = [st[0] for st in steps]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
