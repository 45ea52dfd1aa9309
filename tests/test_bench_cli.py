"""bench.py's command line without a GPU: it measures one GPU only and says
so for any other count, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        res = _bench("--gpus", n)
        assert res.returncode == 2
        assert "one GPU only" in res.stderr
        assert res.stdout == ""


def test_help_lists_the_parts():
    res = _bench("--help")
    assert res.returncode == 0
    for part in ("step", "sweep", "pressure", "msweep", "adjoint", "duct", "pduct"):
        assert part in res.stdout
