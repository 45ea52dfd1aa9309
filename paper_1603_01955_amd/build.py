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

SOURCES = ["clb_api.cpp", "clb_kernels.hip", "clb_batch.hip", "clb_pbatch.hip", "clb_adjoint.hip", "clb_noalloc.hip",
           "clb3d.hip"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
]

# Device pass only: no packed FP32 instructions in device code.  The host
# pass does not know the feature (and would warn for every source), so each
# source is compiled in two passes: the device code object bundle first,
# then the host object with that bundle embedded.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# Host pass only: every host symbol hidden except the C ABI, which
# include/clb.h marks as exported.  No internal function can then be bound at
# run time to a same-named symbol of another loaded object.
HOST_FLAGS = ["-fvisibility=hidden", "-fvisibility-inlines-hidden"]


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
# Sources of the 3-D duct kernels (clb3d.hip and the headers it includes).
DUCT_SOURCES = ["clb3d.hip", "clb_device.hpp", "clb_internal.hpp", "clb_trace.hpp"]


def sources_2d():
    """Every csrc/ file but the 3-D duct's own source."""
    return sorted(f for f in os.listdir(CSRC) if f != "clb3d.hip")


def source_hash(names=STEP_SOURCES):
    """Hash of the given csrc/ files."""
    h = hashlib.sha256()
    for name in sorted(names):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: %s" % " ".join(cmd[-3:]))
    if res.stderr.strip():
        sys.stderr.write(res.stderr)


def _compile(src, objdir, extra_flags, verbose):
    """Device pass (gfx950 code object bundle), then the host object that
    embeds it."""
    base = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0])
    inc = ["-I", INCLUDE, "-I", CSRC]
    common = [hipcc(), "-x", "hip"] + FLAGS + list(extra_flags) + inc
    _run(common + DEVICE_FLAGS + ["--offload-device-only", "-c", src, "-o", base + ".hipfb"], verbose)
    _run(common + HOST_FLAGS + ["--offload-host-only", "-Xclang", "-fcuda-include-gpubinary", "-Xclang",
                                base + ".hipfb", "-c", src, "-o", base + ".o"], verbose)
    return base + ".o"


def build(verbose=False, extra_flags=()):
    import concurrent.futures
    import tempfile
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    with tempfile.TemporaryDirectory(prefix="clb_build_") as objdir:
        workers = max(1, min(len(srcs), os.cpu_count() or 1, 16))
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            objs = list(ex.map(lambda s: _compile(s, objdir, extra_flags, verbose), srcs))
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp] + objs + LINK, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
