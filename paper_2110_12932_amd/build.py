"""Build the HIP/C++ library libtl.so in-tree for gfx950.

Usage: python -m paper_2110_12932_amd.build   (or build() from Python).
The host-side geometry/scan-path unit is compiled by g++ without floating
point contraction; kernels and runtime by hipcc for gfx950 with packed FP32
instructions disabled.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libtl.so")
ARCH = os.environ.get("TL_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if err:
        sys.stderr.write(err + "\n")


def build(verbose=False):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    o = os.path.join(bdir, "tl_host.o")
    _run(["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall",
          "-c", "tl_host.cpp", "-o", o])
    objs.append(o)
    for src in ("tl_kernels.hip", "tl_runtime.cpp", "tl_server.cpp"):
        o = os.path.join(bdir, src.split(".")[0] + ".o")
        extra = ["-x", "hip"] if src.endswith(".cpp") else []
        _run([hipcc] + HIP_FLAGS + [f"-I{INCLUDE}"] + extra + ["-c", src, "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
