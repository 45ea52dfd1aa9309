"""Thin ctypes binding of the 3-D duct step of ``libclb.so`` (the C ABI
declared in include/clb3d.h).  Argument marshalling only: the step runs in
the library's HIP kernels; PyTorch provides device memory and the stream."""
import ctypes
import math

import torch

from . import clb

CLB3_Z_WALLS, CLB3_Z_PERIODIC = 0, 1


class clb3_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("zbc", ctypes.c_int32), ("init", ctypes.c_int32), ("cbbsr_shift", ctypes.c_int32),
        ("xbc", ctypes.c_int32),
        ("kn", ctypes.c_double), ("a", ctypes.c_double), ("sigma", ctypes.c_double),
        ("A1", ctypes.c_double), ("A2", ctypes.c_double), ("r", ctypes.c_double),
        ("s_b", ctypes.c_double), ("s8", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double),
        ("rho0", ctypes.c_double), ("init_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("tq_den", ctypes.c_double), ("p_ratio", ctypes.c_double), ("rho_out", ctypes.c_double),
    ]


_P = ctypes.POINTER(clb3_params)
_SIGNATURES3 = {
    "clb3_params_default": (None, [_P]),
    "clb3_derive": (ctypes.c_int, [_P, ctypes.POINTER(clb.clb_derived)]),
    "clb3_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "clb3_init": (ctypes.c_int, [_P, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "clb3_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "clb3_set_graph_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "clb3_steps_done": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "clb3_moments": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "clb3_massflow": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "clb3_pressure_deviation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "clb3_flow_rate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "clb3_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb3_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb3_check_finite": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "clb3_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}
clb._SIGNATURES.update(_SIGNATURES3)


def lib():
    handle = clb.lib()
    for name, (res, args) in _SIGNATURES3.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    return handle


def make_params3(nx, ny, nz, zbc="walls", kn=0.1, a=2.0, sigma=1.0, A1=None, A2=0.55, r=None, s_b=1.1, s8=1.2,
                 gx=0.0, gy=0.0, gz=0.0, rho0=1.0, init="uniform", init_amp=0.0, seed=0, tq_den=16.0,
                 cbbsr_shift=1, xbc="periodic", p_ratio=2.0, rho_out=1.0):
    p = clb3_params()
    lib().clb3_params_default(ctypes.byref(p))
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.zbc = {"walls": CLB3_Z_WALLS, "periodic": CLB3_Z_PERIODIC}[zbc] if isinstance(zbc, str) else int(zbc)
    p.init = {"uniform": clb.INIT_UNIFORM, "perturbed": clb.INIT_PERTURBED,
              "linear_rho": clb.INIT_LINEAR_RHO}[init] if isinstance(init, str) else int(init)
    p.xbc = {"periodic": clb.X_PERIODIC, "pressure": clb.X_PRESSURE}[xbc] if isinstance(xbc, str) else int(xbc)
    p.p_ratio, p.rho_out = float(p_ratio), float(rho_out)
    p.cbbsr_shift = int(cbbsr_shift)
    p.kn, p.a, p.sigma = float(kn), float(a), float(sigma)
    p.A1 = math.nan if A1 is None else float(A1)
    p.A2 = float(A2)
    p.r = math.nan if r is None else float(r)
    p.s_b, p.s8 = float(s_b), float(s8)
    p.gx, p.gy, p.gz = float(gx), float(gy), float(gz)
    p.rho0, p.init_amp, p.seed = float(rho0), float(init_amp), int(seed)
    p.tq_den = float(tq_den)
    return p


def derive3(params):
    d = clb.clb_derived()
    clb.check(lib().clb3_derive(ctypes.byref(params), ctypes.byref(d)))
    return {"A1": d.A1, "r": d.r, "tau_tilde": d.tau_tilde, "s_nu": d.s_nu, "s_q": d.s_q}


def workspace_size3(params):
    n = ctypes.c_size_t()
    clb.check(lib().clb3_workspace_size(ctypes.byref(params), ctypes.byref(n)))
    return n.value


class Duct:
    """Force-driven or pressure-driven flow in a rectangular microduct (or a
    z-periodic channel), D3Q27 cascaded step; populations live in a torch-allocated
    device workspace, every call enqueues on the current torch stream."""

    def __init__(self, params=None, device="cuda", stream=None, **kw):
        self.params = params if params is not None else make_params3(**kw)
        p = self.params
        self.nx, self.ny, self.nz = p.nx, p.ny, p.nz
        self.device = torch.device(device)
        self.derived = derive3(p)
        nbytes = workspace_size3(p)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        clb.check(lib().clb3_init(ctypes.byref(p), clb._ptr(self.workspace), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx

    def step(self, n=1):
        clb.check(lib().clb3_step(self._ctx, int(n)))
        return self

    def set_graph_steps(self, steps):
        """Replay recorded hipGraphs of `steps` steps (0: launch directly)."""
        clb.check(lib().clb3_set_graph_steps(self._ctx, int(steps)))
        return self

    @property
    def steps_done(self):
        v = ctypes.c_int64()
        clb.check(lib().clb3_steps_done(self._ctx, ctypes.byref(v)))
        return v.value

    def _empty(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def populations(self):
        out = self._empty(27, self.nz, self.ny, self.nx)
        clb.check(lib().clb3_get_populations(self._ctx, clb._ptr(out)))
        return out

    def set_populations(self, P):
        P = P.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(P.shape) != (27, self.nz, self.ny, self.nx):
            raise ValueError("populations must have shape (27, nz, ny, nx)")
        clb.check(lib().clb3_set_populations(self._ctx, clb._ptr(P)))
        self._keep = P

    def moments(self):
        rho, ux, uy, uz = (self._empty(self.nz, self.ny, self.nx) for _ in range(4))
        clb.check(lib().clb3_moments(self._ctx, clb._ptr(rho), clb._ptr(ux), clb._ptr(uy), clb._ptr(uz)))
        return rho, ux, uy, uz

    def massflow(self):
        """(m(x) per cross-section, device tensor [nx]; its mean over x)."""
        m = self._empty(self.nx)
        mean = ctypes.c_double()
        clb.check(lib().clb3_massflow(self._ctx, clb._ptr(m), ctypes.byref(mean)))
        return m, mean.value

    def pressure_deviation(self):
        """(dp(x), rho_c(x)) along the centre line, device tensors [nx]."""
        dp, rc = self._empty(self.nx), self._empty(self.nx)
        clb.check(lib().clb3_pressure_deviation(self._ctx, clb._ptr(dp), clb._ptr(rc)))
        return dp, rc

    def flow_rate(self):
        q = ctypes.c_double()
        clb.check(lib().clb3_flow_rate(self._ctx, ctypes.byref(q)))
        return q.value

    def check_finite(self):
        ok = ctypes.c_int32()
        st = lib().clb3_check_finite(self._ctx, ctypes.byref(ok))
        if st not in (clb.CLB_OK, clb.CLB_EUNSTABLE):
            clb.check(st)
        return bool(ok.value)

    def close(self):
        if getattr(self, "_ctx", None):
            clb.check(lib().clb3_destroy(self._ctx))
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
