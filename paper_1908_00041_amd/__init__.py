"""MI355X (gfx950) forward and adjoint vector spherical harmonic transforms
(FaVeST, Le Gia, Li and Wang).

The transforms run in hand-written HIP kernels behind the C interface of
include/vsht.h (libvsht.so, built in-tree by ``paper_1908_00041_amd.build``);
this package only marshals arguments.  PyTorch provides device memory and
streams.
"""
from ._binding import (EXPORTED, LIB_PATH, PRECISIONS, Plan, VshtError, load_library,
                       vsht_adjoint, vsht_forward, vsht_forward_unweighted, vsht_num_coeffs,
                       vsht_plan, vsht_plan_destroy, vsht_plan_info)

__all__ = ["Plan", "VshtError", "load_library", "vsht_num_coeffs", "vsht_plan", "vsht_forward",
           "vsht_forward_unweighted", "vsht_adjoint", "vsht_plan_info", "vsht_plan_destroy",
           "EXPORTED", "LIB_PATH", "PRECISIONS"]
