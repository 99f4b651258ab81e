"""MI355X (gfx950) hot path of the energy-adaptive Riemannian CG method.

The compute path lives in ``libeahp.so`` (hand-written HIP kernels behind the
C ABI declared in ``include/eahp.h``); this package is a thin ctypes binding
that marshals torch device tensors and host descriptions to that ABI.
"""
from .binding import (EAHP_EARCG, EAHP_EARGD, EAHP_FP64, EAHP_L2RCG, EAHP_MIXED, EAHP_POLAR, EAHP_QR, EahpError, Problem, Server,
                      SolveParams, Stats, frame_from_blocks, frame_to_blocks, layout_estimate, library_path,
                      load_library)

__all__ = ["Problem", "Server", "layout_estimate", "SolveParams", "Stats", "EahpError", "EAHP_FP64", "EAHP_MIXED",
           "EAHP_EARCG", "EAHP_EARGD", "EAHP_L2RCG", "EAHP_POLAR", "EAHP_QR", "load_library", "library_path", "frame_to_blocks",
           "frame_from_blocks"]
