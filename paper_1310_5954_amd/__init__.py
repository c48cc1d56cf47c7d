"""MI355X (gfx950) local ETKF: HIP kernels behind a C ABI (include/letkf.h).

``Filter`` drives one resident ensemble frame by frame; ``Server`` batches the
frames of several resident instances.  The HIP library is loaded on first
use and must have been built (``python -m paper_1310_5954_amd.build``).
"""
from ._lib import BF16, FP32, FP64, LetkfError, build_id, lib
from .api import Filter, Instance, Problem, Server

__all__ = ["BF16", "FP32", "FP64", "LetkfError", "build_id", "lib", "Filter", "Instance", "Problem", "Server"]
