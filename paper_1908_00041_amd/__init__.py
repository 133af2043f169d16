"""MI355X (gfx950) forward and adjoint vector spherical harmonic transforms
(FaVeST, Le Gia, Li and Wang).

The transforms run in hand-written HIP kernels behind the C interface of
include/vsht.h (libvsht.so, built in-tree by ``paper_1908_00041_amd.build``);
this package only marshals arguments.  PyTorch provides device memory and
streams.
"""
from ._binding import (EXPORTED, LIB_PATH, PRECISIONS, BatchPlan, Plan, VshtError, load_library,
                       vsht_adjoint, vsht_forward, vsht_forward_unweighted, vsht_forward_static,
                       vsht_num_coeffs,
                       vsht_plan, vsht_plan_destroy, vsht_plan_info, vsht_forward_many,
                       vsht_adjoint_many, vsht_num_sht_coeffs, vsht_sht_forward,
                       vsht_sht_adjoint, VSHT_UNIT_WEIGHTS, VSHT_TIMES_WEIGHTS)

__all__ = ["Plan", "BatchPlan", "VshtError", "load_library", "vsht_num_coeffs", "vsht_plan", "vsht_forward",
           "vsht_forward_unweighted", "vsht_forward_static", "vsht_adjoint", "vsht_plan_info", "vsht_plan_destroy",
           "vsht_forward_many", "vsht_adjoint_many", "vsht_num_sht_coeffs", "vsht_sht_forward",
           "vsht_sht_adjoint", "VSHT_UNIT_WEIGHTS", "VSHT_TIMES_WEIGHTS",
           "EXPORTED", "LIB_PATH", "PRECISIONS", "AdjointVSHT", "ForwardVSHT", "adjoint_vsht",
           "forward_vsht"]


def __getattr__(name):
    # the autograd functions import torch; load them on first use
    if name in ("AdjointVSHT", "ForwardVSHT", "adjoint_vsht", "forward_vsht"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
