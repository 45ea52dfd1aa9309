"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/clb.h, validates parameters with the documented
status codes, and derives the Eq. (18) / Eq. (21) constants like the CPU
reference."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")

clb = pytest.importorskip("paper_1603_01955_amd.clb")

from oracle import clb_ref as C  # noqa: E402


def _declared_symbols():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            with open(os.path.join(HEADER_DIR, fn)) as fh:
                text = fh.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(clb3?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(clb.LIB_PATH):
        pytest.fail("libclb.so is not built (python -m paper_1603_01955_amd.build)")
    return clb.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared_symbols()
    assert "clb_init" in names and "clb_step" in names and "clb_moments" in names
    assert "clb_massflow" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_exports_nothing_but_the_declared_api(lib):
    """The library's dynamic symbol table holds the entry points of
    include/*.h and nothing else of its own: no internal helper may carry an
    exported plain name, which another loaded object defining the same name
    would take over at run time (calls between exported functions of a shared
    library go through its PLT).  Template code of the C++ standard library
    (namespace std, exported by its own headers) and the per-source
    __hip_cuid markers are allowed."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not found")
    out = subprocess.run([nm, "-D", "--defined-only", clb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    declared = set(_declared_symbols())
    extra = []
    for line in out.splitlines():
        name = line.split()[-1]
        if name in declared or name.startswith("__hip_cuid_"):
            continue
        if re.match(r"_ZN?K?St|_ZN9__gnu_cxx", name):
            continue
        extra.append(name)
    assert not extra, extra


def test_defaults_are_section3_values(lib):
    p = clb.clb_params()
    lib.clb_params_default(ctypes.byref(p))
    assert (p.a, p.A2, p.s3, p.s8, p.sigma, p.tq_den) == (2.0, 0.55, 1.1, 1.2, 1.0, 16.0)
    assert math.isnan(p.A1) and math.isnan(p.r)


@pytest.mark.parametrize("nx,ny,kn,sigma,xbc", [
    (4, 32, 0.1, 1.0, "periodic"), (4000, 40, 0.1, 1.0, "pressure"),
    (32768, 2048, 1.0, 1.0, "periodic"), (2000, 20, 0.1, 0.93, "pressure"),
    (50, 50, 2 * 10 / math.sqrt(math.pi), 1.0, "periodic")])
def test_derived_constants_match_reference(lib, nx, ny, kn, sigma, xbc):
    p = clb.make_params(nx, ny, xbc=xbc, kn=kn, sigma=sigma)
    d = clb.derive(p)
    prm = C.Params(nx=nx, ny=ny, kn=kn, sigma=sigma, xbc=xbc)
    A1, r = C.resolved(prm)
    assert d["A1"] == pytest.approx(A1, rel=1e-15)
    assert d["r"] == pytest.approx(r, rel=1e-15)
    assert d["s_nu"] == pytest.approx(C.rate_nu(kn, ny, 2.0), rel=1e-14)
    assert d["s_q"] == pytest.approx(C.rate_q(kn, ny, 2.0, 0.55), rel=1e-14)
    assert d["tau_tilde"] == pytest.approx(C.tau_tilde(kn, ny, 2.0), rel=1e-14)


def test_workspace_size_arithmetic(lib):
    # rows padded to segments of L = min(1024, next power of two >= nx) lanes
    # plus six per-column arrays and the ghost columns [2][9][ny]
    for nx, ny, padded in ((1000, 30, 1024), (4, 32, 4), (77, 13, 128), (4000, 40, 4096)):
        n = clb.workspace_size(clb.make_params(nx, ny))
        assert n >= 2 * 72 * padded * ny + 6 * 8 * nx + 144 * ny
        assert n < 2 * 72 * padded * ny + 6 * 8 * nx + 144 * ny + 64 * 1024


def test_largest_grid(lib):
    """The size limit sits where one launch can no longer enumerate the padded
    nodes in 64-thread blocks (2^37 padded nodes): one row less is accepted
    and its workspace size does not overflow."""
    n = ctypes.c_size_t()
    p = clb.make_params(1 << 20, (1 << 17) - 1)
    assert lib.clb_workspace_size(ctypes.byref(p), ctypes.byref(n)) == clb.CLB_OK
    assert n.value >= 2 * 72 * (1 << 20) * ((1 << 17) - 1)
    p = clb.make_params(1 << 20, 1 << 17)
    assert lib.clb_workspace_size(ctypes.byref(p), ctypes.byref(n)) == clb.CLB_EINVAL
    assert "too large" in lib.clb_last_error().decode()


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -1), ("xbc", 7), ("init", 9), ("kn", 0.0), ("kn", -1.0), ("kn", math.inf),
    ("a", -0.1), ("sigma", 0.0), ("sigma", 2.5), ("A2", -1.0), ("r", 1.5), ("s3", 2.0),
    ("s8", 0.0), ("gx", math.nan), ("p_ratio", 0.0), ("rho_out", -1.0), ("rho0", 0.0),
    ("init_amp", -1e-3), ("tq_den", 0.0), ("cbbsr_shift", 2), ("forcing", 2)])
def test_invalid_parameters_rejected(lib, field, value):
    p = clb.make_params(8, 8)
    setattr(p, field, value)
    d = clb.clb_derived()
    st = lib.clb_derive(ctypes.byref(p), ctypes.byref(d))
    assert st == clb.CLB_EINVAL
    msg = lib.clb_last_error().decode()
    assert field.split("_")[0] in msg or field in msg
    n = ctypes.c_size_t()
    assert lib.clb_workspace_size(ctypes.byref(p), ctypes.byref(n)) == clb.CLB_EINVAL


def test_pressure_mode_rules(lib):
    p = clb.make_params(1, 8, xbc="pressure")
    assert lib.clb_derive(ctypes.byref(p), ctypes.byref(clb.clb_derived())) == clb.CLB_EINVAL
    p = clb.make_params(10, 8, xbc="pressure")
    p.gx = 1e-6
    assert lib.clb_derive(ctypes.byref(p), ctypes.byref(clb.clb_derived())) == clb.CLB_EINVAL
    assert "pressure" in lib.clb_last_error().decode()


def test_null_arguments(lib):
    p = clb.make_params(8, 8)
    assert lib.clb_derive(ctypes.byref(p), None) == clb.CLB_EINVAL
    assert lib.clb_workspace_size(ctypes.byref(p), None) == clb.CLB_EINVAL
    assert lib.clb_step(None, 1) == clb.CLB_EINVAL
    assert lib.clb_set_steps_per_launch(None, 2) == clb.CLB_EINVAL
    assert lib.clb_destroy(None) == clb.CLB_EINVAL
    out = ctypes.c_void_p()
    assert lib.clb_init(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == clb.CLB_EINVAL
    assert lib.clb_init(ctypes.byref(p), ctypes.c_void_p(4096), 16, None, ctypes.byref(out)) == clb.CLB_ENOMEM
    assert out.value is None


def test_hbm_copy_argument_checks(lib):
    """The copy probe rejects sizes that are not whole 16-byte words, NULL
    and misaligned pointers before touching the GPU, and a zero-byte copy is
    a no-op."""
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)
    assert lib.clb_hbm_copy(a, b, 24, None) == clb.CLB_EINVAL
    assert "multiple of 16" in lib.clb_last_error().decode()
    assert lib.clb_hbm_copy(None, b, 32, None) == clb.CLB_EINVAL
    assert lib.clb_hbm_copy(a, None, 32, None) == clb.CLB_EINVAL
    assert lib.clb_hbm_copy(ctypes.c_void_p((1 << 20) + 8), b, 32, None) == clb.CLB_EINVAL
    assert "16-byte aligned" in lib.clb_last_error().decode()
    assert lib.clb_hbm_copy(a, b, 0, None) == clb.CLB_OK


def test_batch_validation(lib):
    """Batched channels are periodic, start from a uniform or perturbed state,
    and the workspace holds at least every channel's populations."""
    Params = clb.clb_params * 3
    ps = Params(clb.make_params(4, 16, kn=0.1, gx=1e-6), clb.make_params(4, 32, kn=1.0, gx=1e-6),
                clb.make_params(2, 8, kn=3.0))
    n = ctypes.c_size_t()
    assert lib.clb_batch_workspace_size(ctypes.c_int32(3), ps, ctypes.byref(n)) == clb.CLB_OK
    assert n.value >= 72 * (4 * 16 + 4 * 32 + 2 * 8)
    assert lib.clb_batch_workspace_size(ctypes.c_int32(0), ps, ctypes.byref(n)) == clb.CLB_EINVAL
    assert lib.clb_batch_workspace_size(ctypes.c_int32(3), ps, None) == clb.CLB_EINVAL
    bad = Params(ps[0], clb.make_params(10, 8, xbc="pressure"), ps[2])
    assert lib.clb_batch_workspace_size(ctypes.c_int32(3), bad, ctypes.byref(n)) == clb.CLB_EINVAL
    assert "periodic" in lib.clb_last_error().decode()
    bad = Params(ps[0], ps[1], clb.make_params(4, 8, init="linear_rho"))
    assert lib.clb_batch_workspace_size(ctypes.c_int32(3), bad, ctypes.byref(n)) == clb.CLB_EINVAL
    bad = Params(ps[0], ps[1], clb.make_params(4, 8, kn=-1.0))
    assert lib.clb_batch_workspace_size(ctypes.c_int32(3), bad, ctypes.byref(n)) == clb.CLB_EINVAL
    out = ctypes.c_void_p()
    assert lib.clb_batch_init(ctypes.c_int32(3), ps, None, ctypes.c_size_t(0), None,
                              ctypes.byref(out)) == clb.CLB_EINVAL
    assert lib.clb_batch_init(ctypes.c_int32(3), ps, ctypes.c_void_p(4096), ctypes.c_size_t(16), None,
                              ctypes.byref(out)) == clb.CLB_ENOMEM
    assert out.value is None
    assert lib.clb_batch_run(None, ctypes.c_int64(10), ctypes.c_int32(0), ctypes.c_double(0.0), None,
                             None) == clb.CLB_EINVAL
    assert lib.clb_batch_check_finite(None, None) == clb.CLB_EINVAL
    assert lib.clb_batch_destroy(None) == clb.CLB_EINVAL


def test_pressure_batch_validation(lib):
    """A pressure batch holds pressure-driven channels of one grid and one
    wall-source shift; its workspace holds two buffers per channel."""
    Params = clb.clb_params * 3
    ps = Params(clb.make_params(300, 10, xbc="pressure", kn=0.05, p_ratio=1.8, sigma=0.93),
                clb.make_params(300, 10, xbc="pressure", kn=0.5, p_ratio=2.0, A2=0.3),
                clb.make_params(300, 10, xbc="pressure", kn=2.0, p_ratio=1.5, init="uniform"))
    n = ctypes.c_size_t()
    assert lib.clb_pbatch_workspace_size(ctypes.c_int32(3), ps, ctypes.byref(n)) == clb.CLB_OK
    assert n.value >= 3 * 2 * 72 * 512 * 10   # rows padded to 512 lanes
    assert lib.clb_pbatch_workspace_size(ctypes.c_int32(0), ps, ctypes.byref(n)) == clb.CLB_EINVAL
    assert lib.clb_pbatch_workspace_size(ctypes.c_int32(3), ps, None) == clb.CLB_EINVAL
    for bad_ch, field in ((clb.make_params(300, 10, kn=0.1, gx=1e-6), "xbc"),
                          (clb.make_params(301, 10, xbc="pressure"), "nx/ny"),
                          (clb.make_params(300, 11, xbc="pressure"), "nx/ny"),
                          (clb.make_params(300, 10, xbc="pressure", cbbsr_shift=0), "cbbsr_shift"),
                          (clb.make_params(300, 10, xbc="pressure", kn=-1.0), "kn")):
        bad = Params(ps[0], bad_ch, ps[2])
        assert lib.clb_pbatch_workspace_size(ctypes.c_int32(3), bad, ctypes.byref(n)) == clb.CLB_EINVAL
        assert lib.clb_last_error().decode().startswith(field)
    out = ctypes.c_void_p()
    assert lib.clb_pbatch_init(ctypes.c_int32(3), ps, None, ctypes.c_size_t(0), None,
                               ctypes.byref(out)) == clb.CLB_EINVAL
    assert lib.clb_pbatch_init(ctypes.c_int32(3), ps, ctypes.c_void_p(4096), ctypes.c_size_t(16), None,
                               ctypes.byref(out)) == clb.CLB_ENOMEM
    assert out.value is None
    assert lib.clb_pbatch_step(None, ctypes.c_int64(1)) == clb.CLB_EINVAL
    assert lib.clb_pbatch_set_steps_per_launch(None, ctypes.c_int32(2)) == clb.CLB_EINVAL
    assert lib.clb_pbatch_set_path(None, ctypes.c_int32(1)) == clb.CLB_EINVAL
    assert lib.clb_pbatch_check_finite(None, None) == clb.CLB_EINVAL
    assert lib.clb_pbatch_set_populations(None, ctypes.c_int32(0), None) == clb.CLB_EINVAL
    assert lib.clb_pbatch_run(None, ctypes.c_int64(10), ctypes.c_int32(0), ctypes.c_double(0.0), None,
                              None) == clb.CLB_EINVAL
    assert lib.clb_pbatch_massflow(None, None, None) == clb.CLB_EINVAL
    assert lib.clb_pbatch_get_populations(None, ctypes.c_int32(0), None) == clb.CLB_EINVAL
    assert lib.clb_pbatch_destroy(None) == clb.CLB_EINVAL


def test_adjoint_validation(lib):
    """The adjoint covers the pressure-driven channel, T >= 1, 1 <= K <= T;
    its workspace holds the checkpoints and two recompute sets."""
    p = clb.make_params(200, 10, xbc="pressure", kn=0.1, p_ratio=2.0)
    n = ctypes.c_size_t()
    assert lib.clb_adjoint_workspace_size(ctypes.byref(p), ctypes.c_int32(100), ctypes.c_int32(10),
                                          ctypes.byref(n)) == clb.CLB_OK
    state = 72 * 256 * 10                     # one state buffer, rows padded to 256 lanes
    assert n.value >= (10 + 2 * 9 + 4) * state
    for T, K in ((0, 1), (10, 0), (10, 11)):
        assert lib.clb_adjoint_workspace_size(ctypes.byref(p), ctypes.c_int32(T), ctypes.c_int32(K),
                                              ctypes.byref(n)) == clb.CLB_EINVAL
    q = clb.make_params(200, 10, kn=0.1)
    assert lib.clb_adjoint_workspace_size(ctypes.byref(q), ctypes.c_int32(10), ctypes.c_int32(2),
                                          ctypes.byref(n)) == clb.CLB_EINVAL
    assert "pressure" in lib.clb_last_error().decode()
    out = ctypes.c_void_p()
    assert lib.clb_adjoint_init(ctypes.byref(p), ctypes.c_int32(10), ctypes.c_int32(2), None,
                                ctypes.c_size_t(0), None, ctypes.byref(out)) == clb.CLB_EINVAL
    assert lib.clb_adjoint_init(ctypes.byref(p), ctypes.c_int32(10), ctypes.c_int32(2), ctypes.c_void_p(4096),
                                ctypes.c_size_t(16), None, ctypes.byref(out)) == clb.CLB_ENOMEM
    assert out.value is None
    g = (ctypes.c_double * 4)()
    assert lib.clb_adjoint_forward(None, None, ctypes.c_double(1.0), None) == clb.CLB_EINVAL
    assert lib.clb_adjoint_backward(None, g) == clb.CLB_EINVAL
    assert lib.clb_adjoint_destroy(None) == clb.CLB_EINVAL
