"""Build the HIP library libcutmg.so in-tree for gfx950 (MI355X).

Host set-up files are compiled as plain C++ with OpenMP, the kernels with
hipcc for gfx950, and everything is linked into one shared library next to
this file.  Always rebuilds.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcutmg.so")

HOST_SOURCES = ["basis_linalg.cpp", "quadrature.cpp", "setup.cpp", "api.cpp", "server.cpp"]
DEVICE_SOURCES = ["kernels.hip"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile and link libcutmg.so to `out`; `defines` are extra -D flags for
    every source (tuning switches)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="cutmg_build_") as tmp:
        objs = []
        procs = []
        for src in HOST_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            # no FMA contraction on the host: quadrature decisions (box classification,
            # subdivision) then round like the plain IEEE arithmetic of the checking code
            cmd = [hipcc, "-x", "c++", *COMMON, "-ffp-contract=off", "-fopenmp", "-D__HIP_PLATFORM_AMD__",
                   "-I/opt/rocm/include", *[f"-D{d}" for d in defines], "-c",
                   os.path.join(SRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        for src in DEVICE_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc, *COMMON, *HIP_FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(SRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        for cmd, p in procs:
            so, se = p.communicate()
            if p.returncode != 0:
                sys.stderr.write(" ".join(cmd) + "\n" + so + se)
                raise RuntimeError(f"compile failed: {cmd[-3]}")
            if verbose and (so or se):
                sys.stderr.write(so + se)
        tmp_lib = out + ".tmp"
        _run([hipcc, *HIP_FLAGS, "-shared", "-fopenmp", *objs, "-o", tmp_lib])
        os.replace(tmp_lib, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
