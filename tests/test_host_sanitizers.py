"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds a copy of the C ABI library with the host side instrumented
(``-Xarch_host`` before each ``-fsanitize=``; device code is compiled as
usual and never runs here) and links ``host_checks.cpp`` against it.  That
program calls every entry point family with invalid parameters and null
arguments, all of which return before any device work, so the whole run
needs no GPU.  A sanitizer report or a failed expectation fails the test.
"""
import os
import shutil
import subprocess

import pytest

from paper_1603_01955_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
CLANG = "/opt/rocm/llvm/bin/clang++"

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _tools():
    hipcc = B.hipcc()
    if shutil.which(hipcc) is None and not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not found")
    return hipcc


def _run(cmds, cwd):
    """Run the commands concurrently; fail with the output of the first error."""
    procs = [subprocess.Popen(c, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
             for c in cmds]
    outs = [p.communicate(timeout=600)[0] for p in procs]
    for c, p, out in zip(cmds, procs, outs):
        assert p.returncode == 0, "%s\n%s" % (" ".join(c), out[-4000:])


def test_host_code_under_asan_ubsan(tmp_path):
    hipcc = _tools()
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", B.INCLUDE, "-I", B.CSRC] + SAN
    objs, cmds = [], []
    for src in B.SOURCES:
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        cmds.append([hipcc, "-x", "hip"] + common + ["-c", os.path.join(B.CSRC, src), "-o", obj])
    _run(cmds, str(tmp_path))

    lib = str(tmp_path / "libclb_san.so")
    _run([[hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN + objs + ["-o", lib] + B.LINK], str(tmp_path))

    exe = str(tmp_path / "host_checks")
    _run([[CLANG, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-I", B.INCLUDE, os.path.join(HERE, "host_checks.cpp"),
           lib, "-Wl,-rpath," + str(tmp_path), "-o", exe]], str(tmp_path))

    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    res = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "host checks ok" in res.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
