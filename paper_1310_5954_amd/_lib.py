"""ctypes declarations of the C ABI in include/letkf.h.

Argument marshalling only: every step of the filter runs in the HIP library.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libletkf.so")

OK, EINVAL, ENOMEM, EAGAIN, EDEVICE, ENUMERIC, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16 = 0, 1, 2
FLAG_DEBUG = 0x1
FLAG_PISTONS = 0x2
FLAG_GRAPH = 0x4
FLAG_FP32_ROTATIONS = 0x8
SERVER_CLASSES = 16
SERVER_GRAPHS = 0x1
ORDER_MAP, ORDER_COST, ORDER_XCD, ORDER_BALANCED = 0, 1, 2, 3
ORDER_NAMES = {ORDER_MAP: "map", ORDER_COST: "cost", ORDER_XCD: "xcd", ORDER_BALANCED: "balanced"}


class Dims(C.Structure):
    _fields_ = [("n_act", C.c_int32), ("n_sub", C.c_int32), ("m", C.c_int32)]


class Model(C.Structure):
    _fields_ = [("a1", C.POINTER(C.c_double)), ("a2", C.POINTER(C.c_double)),
                ("sigma_v", C.c_double), ("r_inv", C.POINTER(C.c_double)),
                ("d_nnz", C.c_int32), ("d_rowptr", C.POINTER(C.c_int32)),
                ("d_col", C.POINTER(C.c_int32)), ("d_val", C.POINTER(C.c_double)),
                ("inflation", C.c_double), ("seed", C.c_uint64), ("obs_instant", C.c_int32)]


class DomainMapC(C.Structure):
    _fields_ = [("n_domains", C.c_int32), ("est_ptr", C.POINTER(C.c_int32)),
                ("est_act", C.POINTER(C.c_int32)), ("est_w", C.POINTER(C.c_double)),
                ("obs_ptr", C.POINTER(C.c_int32)), ("obs_sub", C.POINTER(C.c_int32)),
                ("obs_taper", C.POINTER(C.c_double))]


class Tuning(C.Structure):
    _fields_ = [("grid", C.c_int32), ("order", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("candidates", C.c_int32), ("best_us", C.c_float), ("default_us", C.c_float)]

    def as_dict(self) -> dict:
        return dict(grid=self.grid, order=ORDER_NAMES.get(self.order, self.order), blocks_per_cu=self.blocks_per_cu,
                    candidates=self.candidates, best_us=round(self.best_us, 2), default_us=round(self.default_us, 2))


DONE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_uint64, C.c_int)

_lib = None


class LetkfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _sig(lib):
    P = C.c_void_p
    pd = C.POINTER(C.c_double)
    lib.letkf_workspace_size.argtypes = [C.POINTER(Dims), C.POINTER(Model), C.POINTER(DomainMapC), C.c_int,
                                         C.c_uint32, C.POINTER(C.c_size_t)]
    lib.letkf_create.argtypes = [C.POINTER(Dims), C.POINTER(Model), C.POINTER(DomainMapC), C.c_int, C.c_uint32,
                                 pd, P, C.c_size_t, P, C.POINTER(P)]
    lib.letkf_destroy.argtypes = [P]
    lib.letkf_analyse.argtypes = [P, P, C.c_int, pd, P]
    lib.letkf_forecast.argtypes = [P, P]
    lib.letkf_step.argtypes = [P, P, C.c_int, pd, P]
    lib.letkf_step_noalloc.argtypes = [P, P, P, P]
    lib.letkf_get_state.argtypes = [P, pd, C.POINTER(C.c_uint64), P]
    lib.letkf_set_state.argtypes = [P, pd, C.c_uint64, P]
    lib.letkf_debug_domain.argtypes = [P, C.c_int32, pd, pd, pd, C.POINTER(C.c_int32), pd, P]
    lib.letkf_debug_placement.argtypes = [P, C.c_int32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                          C.POINTER(C.c_int32), pd, P]
    lib.letkf_debug_substeps.argtypes = [P, C.c_int32, pd, P]
    lib.letkf_unconverged_domains.argtypes = [P, C.POINTER(C.c_int32), P]
    lib.letkf_kernel_times.argtypes = [P, C.c_int, pd, C.POINTER(C.c_uint64)]
    lib.letkf_sweep_stats.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), P]
    lib.letkf_autotune.argtypes = [P, C.c_int32, C.POINTER(Tuning), P]
    lib.letkf_server_autotune.argtypes = [P, C.c_int32, C.POINTER(Tuning)]
    lib.letkf_set_tuning.argtypes = [P, C.POINTER(Tuning), P]
    lib.letkf_last_means.argtypes = [P, pd, pd, P]
    lib.letkf_server_set_tuning.argtypes = [P, C.c_int32, C.POINTER(Tuning)]
    lib.letkf_server_create.argtypes = [P, C.c_size_t, C.c_int32, C.c_uint32, C.POINTER(P)]
    lib.letkf_server_add.argtypes = [P, C.POINTER(Dims), C.POINTER(Model), C.POINTER(DomainMapC), C.c_int,
                                     C.c_uint32, pd, C.POINTER(P)]
    lib.letkf_server_remove.argtypes = [P, P]
    lib.letkf_submit_frame.argtypes = [P, pd, C.c_uint64, pd, DONE_FN, P]
    lib.letkf_submit_frame_device.argtypes = [P, P, C.c_uint64, pd, DONE_FN, P]
    lib.letkf_server_drain.argtypes = [P]
    lib.letkf_server_set_window.argtypes = [P, C.c_uint32]
    lib.letkf_server_stats.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    lib.letkf_server_destroy.argtypes = [P]
    lib.letkf_server_reserved_bytes.argtypes = []
    lib.letkf_server_reserved_bytes.restype = C.c_size_t
    lib.letkf_strerror.argtypes = [C.c_int]
    lib.letkf_strerror.restype = C.c_char_p
    lib.letkf_last_error.argtypes = []
    lib.letkf_last_error.restype = C.c_char_p
    lib.letkf_build_id.argtypes = []
    lib.letkf_build_id.restype = C.c_char_p
    for name in ("letkf_workspace_size", "letkf_create", "letkf_destroy", "letkf_analyse", "letkf_forecast",
                 "letkf_step", "letkf_get_state", "letkf_set_state", "letkf_debug_domain", "letkf_debug_placement", "letkf_debug_substeps",
                 "letkf_unconverged_domains", "letkf_kernel_times", "letkf_sweep_stats", "letkf_autotune",
                 "letkf_server_autotune", "letkf_set_tuning", "letkf_server_set_tuning", "letkf_last_means",
                 "letkf_server_create", "letkf_server_add", "letkf_server_remove",
                 "letkf_submit_frame", "letkf_submit_frame_device", "letkf_server_drain", "letkf_server_set_window", "letkf_server_stats", "letkf_server_destroy"):
        getattr(lib, name).restype = C.c_int


def lib() -> C.CDLL:
    """The loaded HIP library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is missing: build it with "
                              "`python -m paper_1310_5954_amd.build` (no CPU fallback exists)")
        _lib = C.CDLL(LIB_PATH)
        _sig(_lib)
        _check_fresh(_lib)
    return _lib


def _check_fresh(handle) -> None:
    """Refuse a library built from other sources than the ones in this tree."""
    from .build import source_hash
    built = handle.letkf_build_id().decode()
    want = source_hash()
    if built != want:
        raise ImportError(f"{LIB_PATH} was built from sources {built} but the tree holds {want}: "
                          "rebuild with `python -m paper_1310_5954_amd.build`")


def build_id() -> str:
    return lib().letkf_build_id().decode()


def check(status: int, where: str) -> None:
    if status != OK:
        raise LetkfError(status, where, lib().letkf_last_error().decode(errors="replace"))
