"""Build the gfx950 shared library ``libclb.so`` in-tree with hipcc.

Usage: ``python -m paper_1603_01955_amd.build`` (or ``build()`` from Python).
Cross-compiles without a GPU.
"""
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libclb.so")

SOURCES = ["clb_api.cpp", "clb_kernels.hip", "clb_batch.hip", "clb_pbatch.hip", "clb_adjoint.hip"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# roctx ranges around the entry points (rocprofv3 --marker-trace)
LINK = ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


# Sources that define the single-channel step kernels (ties recorded
# profile data to the kernel version it was measured on).
STEP_SOURCES = ["clb_device.hpp", "clb_gather.hpp", "clb_internal.hpp", "clb_kernels.hip"]


def source_hash(names=STEP_SOURCES):
    """Hash of the given csrc/ files."""
    h = hashlib.sha256()
    for name in sorted(names):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def build(verbose=False, extra_flags=()):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-x", "hip"] + FLAGS + list(extra_flags) + ["-I", INCLUDE, "-I", CSRC, "-o", tmp] + srcs + LINK
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % LIB)
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
