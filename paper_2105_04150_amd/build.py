"""Compile the HIP library ``libpdmi.so`` in-tree for gfx950.

Usage: ``python -m paper_2105_04150_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdmi.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# Packed FP32 instructions are kept out of the device code.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"build step failed ({r.returncode}): {cmd[0]}")
    return r.stdout


KERNEL_SOURCES = ("pdmi_step_sliced.hip", "pdmi_step_staged_f64.hip", "pdmi_step_staged_f32.hip",
                  "pdmi_kernels.hip", "pdmi_adjoint.hip", "pdmi_osb.hip")
HOST_SOURCES = ("pdmi_layout.cpp", "pdmi_upload.cpp", "pdmi_run.cpp", "pdmi_api.cpp", "pdmi_api_state.cpp",
                "pdmi_api_adjoint.cpp")


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, cmds = [], []
    for src in KERNEL_SOURCES:
        o = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        objs.append(o)
        cmds.append(["hipcc", "-c", "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *NO_PACKED_FP32,
                     "-munsafe-fp-atomics", os.path.join(CSRC, src), "-o", o])
    for src in HOST_SOURCES:
        o = os.path.join(BUILD_DIR, src.replace(".cpp", ".o"))
        objs.append(o)
        cmds.append(["hipcc", "-c", "-x", "c++", *COMMON, "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                     "-I", os.path.join(ROCM, "include"), os.path.join(CSRC, src), "-o", o])
    with ThreadPoolExecutor(len(cmds)) as ex:
        out = "".join(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    out += _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print(out)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
