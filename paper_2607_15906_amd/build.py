"""Build libgocp.so in-tree: host C++ with g++, HIP sources with hipcc for gfx950.

Usage: ``python -m paper_2607_15906_amd.build`` (or ``build()`` from Python).
Objects go to ``_build/`` at the repository root; the shared library is
written next to this file.  ``--phase-trace`` builds the measurement variant
``libgocp_trace.so`` instead (GOCP_PHASE_TRACE defined: the energy+screen
launch records its phase timestamps; objects in ``_build/trace``).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgocp.so")

HOST_SOURCES = ["host_mapping.cpp", "host_gocp.cpp", "capi_host.cpp"]
HIP_SOURCES = ["kernels.hip", "runtime.hip", "adapt.hip", "serve.hip", "reopt.hip"]

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]
# Packed FP32 instructions stay disabled in every HIP compilation.  Kernel
# arguments are preloaded into scalar registers at wave launch (the code
# object keeps the fallback that loads them when the firmware does not).
HIP_FLAGS = COMMON + [f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
                      "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-kernarg-preload-count=8",
                      "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "unknown target feature" not in l.lower())
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, phase_trace: bool = False) -> str:
    """Compile every source and link libgocp.so (libgocp_trace.so with
    phase_trace); returns the library path."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    bdir = os.path.join(BUILD, "trace") if phase_trace else BUILD
    lib = os.path.join(PKG, "libgocp_trace.so") if phase_trace else LIB
    hip_flags = HIP_FLAGS + (["-DGOCP_PHASE_TRACE"] if phase_trace else [])
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        _run(["g++", *COMMON, "-Wall", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        out = _run([HIPCC, *hip_flags, "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64", "-lpthread", f"-Wl,-rpath,{ROCM}/lib"])
    shutil.move(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, phase_trace="--phase-trace" in sys.argv))
