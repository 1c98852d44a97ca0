"""Build libsmg.so (HIP kernels for gfx950 + host C++) in the package folder.

    python -m paper_2104_13755_amd.build

Host precompute sources are compiled with g++ -ffp-contract=off (every
rounding step of the geometry code is the one written); HIP sources with
hipcc --offload-arch=gfx950.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libsmg.so")

HOST_SRC = ["ssp.cpp", "hier.cpp", "hier_io.cpp", "assemble_host.cpp"]
HIP_SRC = ["kernels.hip", "api.hip", "batch.hip"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))


def build(verbose=False):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = tempfile.mkdtemp(prefix="smg_build_")
    objs = []
    try:
        for s in HOST_SRC:
            o = os.path.join(tmp, s + ".o")
            _run(["g++", "-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall",
                  "-I" + INC, "-c", os.path.join(CSRC, s), "-o", o])
            objs.append(o)
        for s in HIP_SRC:
            src = os.path.join(CSRC, s)
            if not os.path.exists(src):
                continue
            o = os.path.join(tmp, s + ".o")
            _run([hipcc] + HIP_FLAGS + ["-I" + INC, "-c", src, "-o", o])
            objs.append(o)
        out_tmp = LIB + ".tmp"
        _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out_tmp] + objs)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
