"""MI355X-native EV-FDLB time step (arXiv:2503.15187): HIP kernels for gfx950
behind the C ABI of include/evlb.h, with a thin Python binding."""
from .evlb import (Solver, EvlbError, evlb_params, make_params, lib, strerror,  # noqa: F401
                   evlb_validate, evlb_workspace_bytes, evlb_init, evlb_set_equilibrium,
                   evlb_step, evlb_rhs, evlb_moments, evlb_status, evlb_info, evlb_destroy)
