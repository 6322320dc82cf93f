"""Build libash.so in-tree with hipcc for gfx950.

Usage: python paper_2505_08777_amd/build.py [-v]
(run by path, so that the package, and with it a stale library, is not
imported before the build)
"""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libash.so")

SOURCES = ["host.cpp", "validate.cpp", "batch.cpp", "principal.cpp",
           "kernels.hip"]
# the issue-rate microbenchmarks behind the transforms' issue ceiling
UBENCH_SOURCES = ["ubench.hip"]
UBENCH_LIB = os.path.join(PKG, "libash_ubench.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code: hipcc -O3 would
# otherwise form v_pk_fma/add/mul_f32 from ordinary float code.  Matrix-core
# results are kept in VGPRs (no accumulation-register copies).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-I", INCLUDE, "-I", CSRC]


def _link(sources, lib, objdir, verbose):
    objs = []
    for src in sources:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + FLAGS + (["-x", "hip"] if src.endswith(".hip") else []) \
            + ["-c", os.path.join(CSRC, src), "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    tmp = lib + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
         verbose)
    os.replace(tmp, lib)


def build(verbose=False):
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    _link(SOURCES, LIB, objdir, verbose)
    _link(UBENCH_SOURCES, UBENCH_LIB, objdir, verbose)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    if verbose and out.strip():
        print(out)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
