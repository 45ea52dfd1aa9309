"""MI355X-native cascaded lattice Boltzmann (CLB) method for microchannel gas
flow in the slip and transition regimes (Liu & He, arXiv:1603.01955).

The compute path is the gfx950 HIP library ``libclb.so`` behind the C ABI in
include/clb.h; ``clb`` is its Python binding.
"""
from .clb import (Batch, ClbError, PressureBatch, Solver, derive, lib, make_params, workspace_size,  # noqa: F401
                  CLB_OK, CLB_EINVAL, CLB_ENOMEM, CLB_EHIP, CLB_ESTATE, CLB_EUNSTABLE)
from .adjoint import Adjoint, CLBRunLoss  # noqa: F401,E402
from .clb3d import Duct, make_params3  # noqa: E402,F401
