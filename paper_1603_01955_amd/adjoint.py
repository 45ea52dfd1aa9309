"""Python binding of the hand-written adjoint (clb_adjoint_* in include/clb.h)
and a torch.autograd.Function over it.

Argument marshalling only: the forward run, checkpointing, recompute and the
reverse sweep all run in the library's HIP kernels.
"""
import ctypes
import math

import numpy as np
import torch

from . import clb
from .clb import _ptr, check, lib

_SIGS = {
    "clb_adjoint_workspace_size": (ctypes.c_int, [ctypes.POINTER(clb.clb_params), ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "clb_adjoint_init": (ctypes.c_int, [ctypes.POINTER(clb.clb_params), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "clb_adjoint_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_double)]),
    "clb_adjoint_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_adjoint_observables": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "clb_adjoint_final_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "clb_adjoint_vjp_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "clb_adjoint_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}
clb._SIGNATURES.update(_SIGS)


def _lib():
    L = lib()
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


class Adjoint:
    """Forward run of T steps with ceil(T/K) checkpoints and its adjoint."""

    def __init__(self, params, T, K=None, device="cuda", stream=None):
        L = _lib()
        self.params = params
        self.T = int(T)
        self.K = int(K) if K is not None else max(1, int(math.ceil(math.sqrt(self.T))))
        self.nx, self.ny = params.nx, params.ny
        self.device = torch.device(device)
        n = ctypes.c_size_t()
        check(L.clb_adjoint_workspace_size(ctypes.byref(params), self.T, self.K, ctypes.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(L.clb_adjoint_init(ctypes.byref(params), self.T, self.K, _ptr(self.workspace), n.value,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def forward(self, dp_target, m_target):
        self._dpt = torch.as_tensor(dp_target, dtype=torch.float64).to(self.device).contiguous()
        loss = ctypes.c_double()
        check(_lib().clb_adjoint_forward(self._h, _ptr(self._dpt), float(m_target), ctypes.byref(loss)))
        return loss.value

    def backward(self):
        """Returns (dL/da, dL/dA1, dL/dA2, dL/dr) as a numpy array."""
        g = np.zeros(4, dtype=np.float64)
        check(_lib().clb_adjoint_backward(self._h, g.ctypes.data_as(ctypes.c_void_p)))
        return g

    def observables(self):
        dp = torch.empty(self.nx, dtype=torch.float64, device=self.device)
        m = ctypes.c_double()
        check(_lib().clb_adjoint_observables(self._h, _ptr(dp), ctypes.byref(m)))
        return dp, m.value

    def final_state(self):
        out = torch.empty(9, self.ny, self.nx, dtype=torch.float64, device=self.device)
        check(_lib().clb_adjoint_final_state(self._h, _ptr(out)))
        return out

    def vjp_step(self, P, lam_next):
        P = torch.as_tensor(P, dtype=torch.float64).to(self.device).contiguous()
        lam_next = torch.as_tensor(lam_next, dtype=torch.float64).to(self.device).contiguous()
        out = torch.empty_like(P)
        g = np.zeros(3, dtype=np.float64)
        check(_lib().clb_adjoint_vjp_step(self._h, _ptr(P), _ptr(lam_next), _ptr(out),
                                          g.ctypes.data_as(ctypes.c_void_p)))
        return out, g

    def close(self):
        if getattr(self, "_h", None):
            check(_lib().clb_adjoint_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CLBRunLoss(torch.autograd.Function):
    """loss = CLBRunLoss.apply(theta, spec) with theta = (a, A1, A2, r) a
    float64 tensor and spec a dict: nx, ny, kn (outlet Kn), p_ratio, T, K,
    dp_target (nx), m_target, r_free (bool; if False r follows A1 through
    Eq. 21 and theta[3] is unused), plus optional make_params keywords."""

    @staticmethod
    def forward(ctx, theta, spec):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        extra = {k: v for k, v in spec.items()
                 if k not in ("nx", "ny", "kn", "p_ratio", "T", "K", "dp_target", "m_target", "r_free")}
        params = clb.make_params(spec["nx"], spec["ny"], xbc="pressure", kn=spec["kn"],
                                 p_ratio=spec["p_ratio"], a=th[0], A1=th[1], A2=th[2],
                                 r=th[3] if spec.get("r_free", True) else None, **extra)
        adj = Adjoint(params, spec["T"], spec.get("K"), device=spec.get("device", "cuda"))
        loss = adj.forward(spec["dp_target"], spec["m_target"])
        ctx.adj = adj
        ctx.r_free = spec.get("r_free", True)
        ctx.theta_device = theta.device
        return torch.tensor(loss, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.adj.backward()
        if ctx.r_free:
            g[1] = 0.0          # A1 enters only through r
        else:
            g[3] = 0.0          # r is not an independent parameter
        ctx.adj.close()
        grad = torch.tensor(g, dtype=torch.float64, device=ctx.theta_device)
        return grad_out * grad, None
