"""Thin ctypes binding of ``libclb.so`` (the C ABI declared in include/clb.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory (the workspace and output
arrays) and the stream.  There is no CPU fallback: if the library is not
built, loading it raises.
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclb.so")

CLB_OK, CLB_EINVAL, CLB_ENOMEM, CLB_EHIP, CLB_ESTATE, CLB_EUNSTABLE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "CLB_OK", -1: "CLB_EINVAL", -2: "CLB_ENOMEM", -3: "CLB_EHIP",
                -4: "CLB_ESTATE", -5: "CLB_EUNSTABLE"}
X_PERIODIC, X_PRESSURE = 0, 1
INIT_UNIFORM, INIT_LINEAR_RHO, INIT_PERTURBED = 0, 1, 2


class ClbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class clb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xbc", ctypes.c_int32), ("init", ctypes.c_int32),
        ("kn", ctypes.c_double), ("a", ctypes.c_double), ("sigma", ctypes.c_double),
        ("A1", ctypes.c_double), ("A2", ctypes.c_double), ("r", ctypes.c_double),
        ("s3", ctypes.c_double), ("s8", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("p_ratio", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("rho0", ctypes.c_double), ("ux0", ctypes.c_double), ("uy0", ctypes.c_double),
        ("init_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("tq_den", ctypes.c_double),
        ("cbbsr_shift", ctypes.c_int32), ("forcing", ctypes.c_int32),
    ]


class clb_derived(ctypes.Structure):
    _fields_ = [("A1", ctypes.c_double), ("r", ctypes.c_double), ("tau_tilde", ctypes.c_double),
                ("s_nu", ctypes.c_double), ("s_q", ctypes.c_double)]


_lib = None

_SIGNATURES = {
    "clb_params_default": (None, [ctypes.POINTER(clb_params)]),
    "clb_derive": (ctypes.c_int, [ctypes.POINTER(clb_params), ctypes.POINTER(clb_derived)]),
    "clb_workspace_size": (ctypes.c_int, [ctypes.POINTER(clb_params), ctypes.POINTER(ctypes.c_size_t)]),
    "clb_init": (ctypes.c_int, [ctypes.POINTER(clb_params), ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "clb_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "clb_steps_done": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "clb_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "clb_column_sums": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "clb_massflow": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "clb_flow_rate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "clb_pressure_deviation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "clb_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_check_finite": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "clb_set_check_every": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "clb_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "clb_set_steps_per_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "clb_set_pressure_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "clb_set_graph_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "clb_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "clb_massflow_noalloc": (ctypes.c_int, [ctypes.POINTER(clb_params), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "clb_hbm_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "clb_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libclb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libclb.so not built: run `python -m paper_1603_01955_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status):
    if status != CLB_OK:
        raise ClbError(status, lib().clb_last_error().decode())


def make_params(nx, ny, xbc="periodic", kn=0.1, a=2.0, sigma=1.0, A1=None, A2=0.55, r=None,
                s3=1.1, s8=1.2, gx=0.0, gy=0.0, p_ratio=2.0, rho_out=1.0, rho0=1.0, ux0=0.0,
                uy0=0.0, init=None, init_amp=0.0, seed=0, tq_den=16.0, cbbsr_shift=1, forcing=0):
    p = clb_params()
    lib().clb_params_default(ctypes.byref(p))
    p.nx, p.ny = int(nx), int(ny)
    p.xbc = {"periodic": X_PERIODIC, "pressure": X_PRESSURE}[xbc] if isinstance(xbc, str) else int(xbc)
    if init is None:
        init = INIT_LINEAR_RHO if p.xbc == X_PRESSURE else INIT_UNIFORM
    elif isinstance(init, str):
        init = {"uniform": INIT_UNIFORM, "linear_rho": INIT_LINEAR_RHO, "perturbed": INIT_PERTURBED}[init]
    p.init = int(init)
    p.kn, p.a, p.sigma = float(kn), float(a), float(sigma)
    p.A1 = math.nan if A1 is None else float(A1)
    p.A2 = float(A2)
    p.r = math.nan if r is None else float(r)
    p.s3, p.s8 = float(s3), float(s8)
    p.gx, p.gy = float(gx), float(gy)
    p.p_ratio, p.rho_out = float(p_ratio), float(rho_out)
    p.rho0, p.ux0, p.uy0 = float(rho0), float(ux0), float(uy0)
    p.init_amp, p.seed = float(init_amp), int(seed)
    p.tq_den = float(tq_den)
    p.cbbsr_shift = int(cbbsr_shift)
    p.forcing = int(forcing)
    return p


def derive(params):
    d = clb_derived()
    check(lib().clb_derive(ctypes.byref(params), ctypes.byref(d)))
    return {"A1": d.A1, "r": d.r, "tau_tilde": d.tau_tilde, "s_nu": d.s_nu, "s_q": d.s_q}


def workspace_size(params):
    n = ctypes.c_size_t()
    check(lib().clb_workspace_size(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """One channel: populations live in a torch-allocated device workspace;
    every call enqueues on the current torch stream of ``device``."""

    def __init__(self, params=None, device="cuda", stream=None, **kw):
        self.params = params if params is not None else make_params(**kw)
        self.nx, self.ny = self.params.nx, self.params.ny
        self.device = torch.device(device)
        self.derived = derive(self.params)
        nbytes = workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        check(lib().clb_init(ctypes.byref(self.params), _ptr(self.workspace), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx

    # -- stepping ---------------------------------------------------------
    def step(self, n=1):
        check(lib().clb_step(self._ctx, int(n)))
        return self

    @property
    def steps_done(self):
        v = ctypes.c_int64()
        check(lib().clb_steps_done(self._ctx, ctypes.byref(v)))
        return v.value

    def set_check_every(self, check_every):
        """step() checks for non-finite populations at every multiple of
        check_every steps and raises ClbError (CLB_EUNSTABLE) at the first
        failed check; 0 switches the checks off."""
        check(lib().clb_set_check_every(self._ctx, int(check_every)))

    def set_launch(self, block_x=1024, xcd_remap=1):
        check(lib().clb_set_launch(self._ctx, int(block_x), int(xcd_remap)))

    def set_steps_per_launch(self, steps):
        check(lib().clb_set_steps_per_launch(self._ctx, int(steps)))

    def set_pressure_path(self, path=0):
        """Pressure-mode kernel: 0 by grid size, 1 column kernel, 2 row kernel."""
        check(lib().clb_set_pressure_path(self._ctx, int(path)))

    def set_graph_steps(self, steps_per_graph):
        check(lib().clb_set_graph_steps(self._ctx, int(steps_per_graph)))

    # -- state ------------------------------------------------------------
    def _empty(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def populations(self):
        out = self._empty(9, self.ny, self.nx)
        check(lib().clb_get_populations(self._ctx, _ptr(out)))
        return out

    def set_populations(self, P):
        P = P.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(P.shape) != (9, self.ny, self.nx):
            raise ValueError("populations must have shape (9, ny, nx)")
        check(lib().clb_set_populations(self._ctx, _ptr(P)))
        self._keep = P   # keep alive until the copy on the stream has run

    # -- diagnostics ------------------------------------------------------
    def moments(self):
        rho, ux, uy = (self._empty(self.ny, self.nx) for _ in range(3))
        check(lib().clb_moments(self._ctx, _ptr(rho), _ptr(ux), _ptr(uy)))
        return rho, ux, uy

    def column_sums(self):
        m, su, rc = (self._empty(self.nx) for _ in range(3))
        check(lib().clb_column_sums(self._ctx, _ptr(m), _ptr(su), _ptr(rc)))
        return m, su, rc

    def massflow(self):
        m = self._empty(self.nx)
        mean = ctypes.c_double()
        check(lib().clb_massflow(self._ctx, _ptr(m), ctypes.byref(mean)))
        return m, mean.value

    def flow_rate(self):
        q = ctypes.c_double()
        check(lib().clb_flow_rate(self._ctx, ctypes.byref(q)))
        return q.value

    def pressure_deviation(self):
        dp, rc = self._empty(self.nx), self._empty(self.nx)
        check(lib().clb_pressure_deviation(self._ctx, _ptr(dp), _ptr(rc)))
        return dp, rc

    def check_finite(self):
        ok = ctypes.c_int32()
        st = lib().clb_check_finite(self._ctx, ctypes.byref(ok))
        if st not in (CLB_OK, CLB_EUNSTABLE):
            check(st)
        return bool(ok.value)

    def close(self):
        if getattr(self, "_ctx", None):
            check(lib().clb_destroy(self._ctx))
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def massflow_noalloc(params, P, m_col=None, stream=None):
    """clb_massflow of caller-held populations P ([9][ny][nx] float64 on the
    GPU) with no device allocation: returns the column mean; fills m_col
    ([nx] float64 on the GPU) if given.  Enqueued on ``stream`` (default: the
    current stream of P's device)."""
    if stream is None:
        stream = torch.cuda.current_stream(P.device)
    mean = ctypes.c_double()
    check(lib().clb_massflow_noalloc(ctypes.byref(params), _ptr(P), _ptr(m_col), ctypes.byref(mean),
                                     ctypes.c_void_p(stream.cuda_stream)))
    return mean.value


def hbm_copy(src, dst, stream=None):
    """Plain device copy of src into dst (same byte size, both CUDA tensors),
    the library's HBM ceiling probe, enqueued on ``stream`` (default: the
    current stream of src's device)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    if stream is None:
        stream = torch.cuda.current_stream(src.device)
    check(lib().clb_hbm_copy(_ptr(src), _ptr(dst), nbytes, ctypes.c_void_p(stream.cuda_stream)))


_BATCH_SIGNATURES = {
    "clb_batch_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "clb_batch_init": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "clb_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "clb_batch_flow_rate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_batch_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "clb_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "clb_batch_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "clb_batch_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "clb_batch_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "clb_batch_check_finite": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}
_SIGNATURES.update(_BATCH_SIGNATURES)


def batch_workspace_size(params_list):
    arr = (clb_params * len(params_list))(*params_list)
    n = ctypes.c_size_t()
    check(lib().clb_batch_workspace_size(len(params_list), arr, ctypes.byref(n)))
    return n.value


class Batch:
    """Many independent periodic channels advanced by one persistent launch
    (the Kn sweep of Section 3.1).  ``params_list`` holds one clb_params per
    channel (see make_params)."""

    def __init__(self, params_list, device="cuda", stream=None):
        import numpy as np
        self.params = list(params_list)
        self.nch = len(self.params)
        self.device = torch.device(device)
        self._arr = (clb_params * self.nch)(*self.params)
        nbytes = batch_workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib().clb_batch_init(self.nch, self._arr, _ptr(self.workspace), nbytes,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._steps = np.zeros(self.nch, dtype=np.int64)
        self._conv = np.zeros(self.nch, dtype=np.int32)

    def run(self, max_steps, check_every=0, tol=0.0):
        """Returns (steps per channel, converged flags) as numpy arrays."""
        check(lib().clb_batch_run(self._h, int(max_steps), int(check_every), float(tol),
                                  self._steps.ctypes.data_as(ctypes.c_void_p),
                                  self._conv.ctypes.data_as(ctypes.c_void_p)))
        return self._steps.copy(), self._conv.astype(bool)

    def flow_rate(self):
        import numpy as np
        q = np.zeros(self.nch, dtype=np.float64)
        check(lib().clb_batch_flow_rate(self._h, q.ctypes.data_as(ctypes.c_void_p)))
        return q

    def set_launch(self, threads, longest_first=1):
        check(lib().clb_batch_set_launch(self._h, int(threads), int(longest_first)))

    def tune(self, probe_steps=500):
        t, o = ctypes.c_int32(), ctypes.c_int32()
        check(lib().clb_batch_tune(self._h, int(probe_steps), ctypes.byref(t), ctypes.byref(o)))
        return t.value, o.value

    def populations(self, ch):
        p = self.params[ch]
        out = torch.empty(9, p.ny, p.nx, dtype=torch.float64, device=self.device)
        check(lib().clb_batch_get_populations(self._h, int(ch), _ptr(out)))
        return out

    def set_populations(self, ch, P):
        p = self.params[ch]
        P = P.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(P.shape) != (9, p.ny, p.nx):
            raise ValueError("populations must have shape (9, ny, nx)")
        check(lib().clb_batch_set_populations(self._h, int(ch), _ptr(P)))
        torch.cuda.current_stream(self.device).synchronize()

    def reset(self):
        check(lib().clb_batch_reset(self._h))

    def check_finite(self):
        """Per-channel flags (numpy bool array): True where every population
        is finite.  Does not raise for non-finite channels."""
        import numpy as np
        ok = np.zeros(self.nch, dtype=np.int32)
        st = lib().clb_batch_check_finite(self._h, ok.ctypes.data_as(ctypes.c_void_p))
        if st not in (CLB_OK, CLB_EUNSTABLE):
            check(st)
        return ok.astype(bool)

    def close(self):
        if getattr(self, "_h", None):
            check(lib().clb_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_PBATCH_SIGNATURES = {
    "clb_pbatch_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "clb_pbatch_init": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "clb_pbatch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "clb_pbatch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "clb_pbatch_set_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "clb_pbatch_set_steps_per_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "clb_pbatch_massflow": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "clb_pbatch_column_sums": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "clb_pbatch_pressure_deviation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "clb_pbatch_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "clb_pbatch_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "clb_pbatch_check_finite": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_pbatch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}
_SIGNATURES.update(_PBATCH_SIGNATURES)


def pbatch_workspace_size(params_list):
    arr = (clb_params * len(params_list))(*params_list)
    n = ctypes.c_size_t()
    check(lib().clb_pbatch_workspace_size(len(params_list), arr, ctypes.byref(n)))
    return n.value


class PressureBatch:
    """Many pressure-driven channels of one grid advanced together (the
    mass-flow study of Section 3.2).  ``params_list`` holds one clb_params per
    channel (see make_params, xbc="pressure"); all share nx, ny and
    cbbsr_shift."""

    def __init__(self, params_list, device="cuda", stream=None):
        import numpy as np
        self.params = list(params_list)
        self.nch = len(self.params)
        self.nx, self.ny = self.params[0].nx, self.params[0].ny
        self.device = torch.device(device)
        self._arr = (clb_params * self.nch)(*self.params)
        nbytes = pbatch_workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib().clb_pbatch_init(self.nch, self._arr, _ptr(self.workspace), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._steps = np.zeros(self.nch, dtype=np.int64)
        self._conv = np.zeros(self.nch, dtype=np.int32)

    def step(self, n=1):
        check(lib().clb_pbatch_step(self._h, int(n)))

    def run(self, max_steps, check_every=0, tol=0.0):
        """Returns (steps per channel, converged flags) as numpy arrays."""
        check(lib().clb_pbatch_run(self._h, int(max_steps), int(check_every), float(tol),
                                   self._steps.ctypes.data_as(ctypes.c_void_p),
                                   self._conv.ctypes.data_as(ctypes.c_void_p)))
        return self._steps.copy(), self._conv.astype(bool)

    def set_path(self, path=0):
        """0: by total size, 1: column kernel, 2: row kernel."""
        check(lib().clb_pbatch_set_path(self._h, int(path)))

    def set_steps_per_launch(self, steps=4):
        check(lib().clb_pbatch_set_steps_per_launch(self._h, int(steps)))

    def massflow(self):
        """(m, m_ns): column-mean mass flow of each channel and the continuum
        no-slip mass flow of the same channel; S = m / m_ns."""
        import numpy as np
        m = np.zeros(self.nch, dtype=np.float64)
        mns = np.zeros(self.nch, dtype=np.float64)
        check(lib().clb_pbatch_massflow(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                        mns.ctypes.data_as(ctypes.c_void_p)))
        return m, mns

    def column_sums(self, ch):
        """(m(x), sum_y u_x(x), rho_c(x)) of channel ch, device tensors [nx]."""
        m, su, rc = (torch.empty(self.nx, dtype=torch.float64, device=self.device) for _ in range(3))
        check(lib().clb_pbatch_column_sums(self._h, int(ch), _ptr(m), _ptr(su), _ptr(rc)))
        return m, su, rc

    def pressure_deviation(self, ch):
        dp = torch.empty(self.nx, dtype=torch.float64, device=self.device)
        check(lib().clb_pbatch_pressure_deviation(self._h, int(ch), _ptr(dp)))
        return dp

    def populations(self, ch):
        out = torch.empty(9, self.ny, self.nx, dtype=torch.float64, device=self.device)
        check(lib().clb_pbatch_get_populations(self._h, int(ch), _ptr(out)))
        return out

    def set_populations(self, ch, P):
        P = P.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(P.shape) != (9, self.ny, self.nx):
            raise ValueError("populations must have shape (9, ny, nx)")
        check(lib().clb_pbatch_set_populations(self._h, int(ch), _ptr(P)))
        torch.cuda.current_stream(self.device).synchronize()

    def check_finite(self):
        """Per-channel flags (numpy bool array): True where every population
        is finite.  Does not raise for non-finite channels."""
        import numpy as np
        ok = np.zeros(self.nch, dtype=np.int32)
        st = lib().clb_pbatch_check_finite(self._h, ok.ctypes.data_as(ctypes.c_void_p))
        if st not in (CLB_OK, CLB_EUNSTABLE):
            check(st)
        return ok.astype(bool)

    def close(self):
        if getattr(self, "_h", None):
            check(lib().clb_pbatch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
