"""Python binding of the local ETKF library: one resident filter instance.

Argument marshalling only.  Device memory comes from PyTorch (the workspace
is a uint8 CUDA tensor) and the HIP stream is torch's current stream; every
step of the filter runs in the HIP kernels of libletkf.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

_pd = C.POINTER(C.c_double)
_pi = C.POINTER(C.c_int32)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class Problem:
    """C structs (and the numpy arrays they point into) for one instance."""

    def __init__(self, n_act, n_sub, m, a1, a2, sigma_v, r_inv, d_rowptr, d_col, d_val, est_ptr, est_act,
                 est_w, obs_ptr, obs_sub, obs_taper, inflation=1.0, seed=0, obs_instant=0):
        self.keep = dict(a1=_f64(a1), a2=_f64(a2), r_inv=_f64(r_inv), rowptr=_i32(d_rowptr), col=_i32(d_col),
                         val=_f64(d_val), est_ptr=_i32(est_ptr), est_act=_i32(est_act), est_w=_f64(est_w),
                         obs_ptr=_i32(obs_ptr), obs_sub=_i32(obs_sub), obs_taper=_f64(obs_taper))
        k = self.keep
        self.n_act, self.n_sub, self.m = int(n_act), int(n_sub), int(m)
        self.dims = L.Dims(self.n_act, self.n_sub, self.m)
        self.model = L.Model(k["a1"].ctypes.data_as(_pd), k["a2"].ctypes.data_as(_pd), float(sigma_v),
                             k["r_inv"].ctypes.data_as(_pd), int(len(k["col"])), k["rowptr"].ctypes.data_as(_pi),
                             k["col"].ctypes.data_as(_pi), k["val"].ctypes.data_as(_pd), float(inflation),
                             int(seed) & 0xFFFFFFFFFFFFFFFF, int(obs_instant))
        self.map = L.DomainMapC(int(len(k["est_ptr"]) - 1), k["est_ptr"].ctypes.data_as(_pi),
                                k["est_act"].ctypes.data_as(_pi), k["est_w"].ctypes.data_as(_pd),
                                k["obs_ptr"].ctypes.data_as(_pi), k["obs_sub"].ctypes.data_as(_pi),
                                k["obs_taper"].ctypes.data_as(_pd))

    @classmethod
    def from_case(cls, case, dmap=None, sigma_v=None, seed=None, obs_instant=0):
        dm = dmap if dmap is not None else case.dmap
        return cls(case.n_act, case.n_sub, case.m, case.a1, case.a2,
                   case.sigma_v if sigma_v is None else sigma_v, case.r_inv, case.D.rowptr, case.D.col,
                   case.D.val, dm.est_ptr, dm.est_act, dm.est_w, dm.obs_ptr, dm.obs_sub, dm.obs_taper,
                   case.inflation, case.philox_seed if seed is None else seed, obs_instant)

    @property
    def n(self):
        return 2 * self.n_act

    @property
    def p(self):
        return 2 * self.n_sub

    def workspace_size(self, precision: int, flags: int = 0) -> int:
        b = C.c_size_t()
        L.check(L.lib().letkf_workspace_size(C.byref(self.dims), C.byref(self.model), C.byref(self.map),
                                             precision, flags, C.byref(b)), "letkf_workspace_size")
        return int(b.value)


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Filter:
    """One resident ensemble on the GPU (plain per-frame path)."""

    def __init__(self, problem: Problem, X0, precision: int = L.FP64, debug: bool = False, device="cuda:0",
                 pistons: bool = False, graph: bool = False, fp32_rotations: bool = False):
        self.problem = problem
        self.precision = int(precision)
        self.device = torch.device(device)
        self.flags = ((L.FLAG_DEBUG if debug else 0) | (L.FLAG_PISTONS if pistons else 0)
                      | (L.FLAG_GRAPH if graph else 0) | (L.FLAG_FP32_ROTATIONS if fp32_rotations else 0))
        X0 = _f64(X0)
        if X0.shape != (problem.n, problem.m):
            raise ValueError(f"X0 must be ({problem.n}, {problem.m}), got {X0.shape}")
        nbytes = problem.workspace_size(self.precision, self.flags)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_create(C.byref(problem.dims), C.byref(problem.model), C.byref(problem.map),
                                         self.precision, self.flags, X0.ctypes.data_as(_pd),
                                         C.c_void_p(self.workspace.data_ptr()), nbytes, _stream(self.device),
                                         C.byref(h)), "letkf_create")
        self.handle = h
        self._out = np.empty(problem.n_act)

    def close(self):
        if getattr(self, "handle", None):
            L.lib().letkf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _y(self, y):
        if isinstance(y, torch.Tensor) and y.is_cuda:
            if y.dtype != torch.float64 or not y.is_contiguous() or y.numel() != self.problem.p:
                raise ValueError("device y must be a contiguous float64 tensor of p values")
            return C.c_void_p(y.data_ptr()), 1, y
        a = _f64(y)
        if a.shape != (self.problem.p,):
            raise ValueError(f"y must have {self.problem.p} values")
        return C.c_void_p(a.ctypes.data), 0, a

    def analyse(self, y, mean: bool = False):
        ptr, on_dev, keep = self._y(y)
        out = np.empty(self.problem.n_act) if mean else None
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_analyse(self.handle, ptr, on_dev, out.ctypes.data_as(_pd) if mean else None,
                                          _stream(self.device)), "letkf_analyse")
        return out

    def forecast(self):
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_forecast(self.handle, _stream(self.device)), "letkf_forecast")

    def step(self, y, pred: bool = True):
        ptr, on_dev, keep = self._y(y)
        out = np.empty(self.problem.n_act) if pred else None
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_step(self.handle, ptr, on_dev, out.ctypes.data_as(_pd) if pred else None,
                                       _stream(self.device)), "letkf_step")
        return out

    def get_state(self):
        X = np.empty((self.problem.n, self.problem.m))
        f = C.c_uint64()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_get_state(self.handle, X.ctypes.data_as(_pd), C.byref(f), _stream(self.device)),
                    "letkf_get_state")
        return X, int(f.value)

    def set_state(self, X, frame: int = 0):
        X = _f64(X)
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_set_state(self.handle, X.ctypes.data_as(_pd), int(frame), _stream(self.device)),
                    "letkf_set_state")

    def debug_domain(self, l: int):
        m = self.problem.m
        Cm, lam, T, cyc = np.empty((m, m)), np.empty(m), np.empty((m, m)), np.empty(5)
        sw = C.c_int32()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_debug_domain(self.handle, int(l), Cm.ctypes.data_as(_pd), lam.ctypes.data_as(_pd),
                                               T.ctypes.data_as(_pd), C.byref(sw), cyc.ctypes.data_as(_pd),
                                               _stream(self.device)), "letkf_debug_domain")
        return dict(C=Cm, lam=lam, T=T, sweeps=int(sw.value),
                    cycles=dict(zip(("gather_C", "cholesky", "jacobi", "transform", "update"), cyc.tolist())))

    def debug_placement(self, l: int) -> dict:
        """Where domain l's analysis ran in the last analysis: XCD, shader
        engine, shader array, CU and SIMD (decoded from HW_ID / XCC_ID) and its
        start clock (letkf_debug_placement)."""
        hw, xcc, wg, t0 = C.c_uint32(), C.c_uint32(), C.c_int32(), C.c_double()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_debug_placement(self.handle, int(l), C.byref(hw), C.byref(xcc), C.byref(wg),
                                                  C.byref(t0), _stream(self.device)), "letkf_debug_placement")
        h = hw.value
        return dict(xcd=xcc.value & 0xF, se=(h >> 13) & 0x7, sh=(h >> 12) & 1, cu=(h >> 8) & 0xF,
                    simd=(h >> 4) & 0x3, workgroup=wg.value, start_clock=t0.value)

    def debug_substeps(self, l: int) -> dict:
        """Cycles of the sub-steps of domain l's wbar/W/T phase in the last
        analysis (letkf_debug_substeps)."""
        cyc = np.empty(4)
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_debug_substeps(self.handle, int(l), cyc.ctypes.data_as(_pd), _stream(self.device)),
                    "letkf_debug_substeps")
        return dict(zip(("U", "wbar", "refine", "T"), cyc.tolist()))

    def kernel_times(self, enable: bool):
        """Accumulated kernel milliseconds {slopes, analysis, merge/forecast} and
        the number of timed calls since the last enable; then (re)enables or stops."""
        ms = (C.c_double * 3)()
        n = C.c_uint64()
        L.check(L.lib().letkf_kernel_times(self.handle, 1 if enable else 0, ms, C.byref(n)), "letkf_kernel_times")
        return list(ms), int(n.value)

    def sweep_stats(self):
        sw, so = C.c_uint64(), C.c_uint64()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_sweep_stats(self.handle, C.byref(sw), C.byref(so), _stream(self.device)),
                    "letkf_sweep_stats")
        return int(sw.value), int(so.value)

    def autotune(self, reps: int = 3) -> dict:
        """Times the analysis launch shapes on the resident data and keeps the
        fastest (letkf_autotune); returns the choice and its timings."""
        t = L.Tuning()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_autotune(self.handle, int(reps), C.byref(t), _stream(self.device)),
                    "letkf_autotune")
        return t.as_dict()

    def last_means(self):
        """(analysis mean of phi_k, prediction mean of phi_{k+1}) of the last frame."""
        a, p = np.empty(self.problem.n_act), np.empty(self.problem.n_act)
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_last_means(self.handle, a.ctypes.data_as(_pd), p.ctypes.data_as(_pd),
                                             _stream(self.device)), "letkf_last_means")
        return a, p

    def set_tuning(self, grid: int, order: int = L.ORDER_COST):
        """Applies a launch shape chosen earlier (letkf_set_tuning; order: L.ORDER_*)."""
        t = L.Tuning(grid=int(grid), order=int(order))
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_set_tuning(self.handle, C.byref(t), _stream(self.device)), "letkf_set_tuning")

    def unconverged(self) -> int:
        c = C.c_int32()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_unconverged_domains(self.handle, C.byref(c), _stream(self.device)),
                    "letkf_unconverged_domains")
        return int(c.value)


class Instance:
    """A filter instance resident in a Server's arena."""

    def __init__(self, server, handle, problem, precision):
        self.server = server
        self.handle = handle
        self.problem = problem
        self.precision = precision

    def get_state(self):
        X = np.empty((self.problem.n, self.problem.m))
        f = C.c_uint64()
        L.check(L.lib().letkf_get_state(self.handle, X.ctypes.data_as(_pd), C.byref(f), None), "letkf_get_state")
        return X, int(f.value)

    def set_state(self, X, frame: int = 0):
        X = _f64(X)
        L.check(L.lib().letkf_set_state(self.handle, X.ctypes.data_as(_pd), int(frame), None), "letkf_set_state")


class Server:
    """Continuous-batching frame server over resident instances.

    The HBM budget is a uint8 CUDA tensor of ``budget_bytes`` handed to the
    library as its arena.  ``submit`` returns at once; completion is reported
    through ``done`` (frame_id -> (status, perf_counter time)) and the
    caller's prediction buffer is filled before the frame is marked done."""

    def __init__(self, budget_bytes: int, max_batch: int = 64, device="cuda:0", on_done=None, graphs: bool = False):
        self.device = torch.device(device)
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        self.done = {}
        self.on_done = on_done          # optional hook(frame_id, status, time), runs on the completion thread
        self._keep = {}
        self._cb = L.DONE_FN(self._on_done)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            torch.cuda.synchronize(self.device)
            L.check(L.lib().letkf_server_create(C.c_void_p(self.arena.data_ptr()), int(budget_bytes), int(max_batch),
                                                L.SERVER_GRAPHS if graphs else 0, C.byref(h)), "letkf_server_create")
        self.handle = h

    def _on_done(self, user, frame_id, status):
        import time
        t = time.perf_counter()
        self.done[int(frame_id)] = (int(status), t)
        self._keep.pop(int(frame_id), None)
        if self.on_done is not None:
            self.on_done(int(frame_id), int(status), t)

    def add(self, problem: Problem, X0, precision: int = L.FP64, pistons: bool = False,
            fp32_rotations: bool = False) -> Instance:
        X0 = _f64(X0)
        h = C.c_void_p()
        flags = (L.FLAG_PISTONS if pistons else 0) | (L.FLAG_FP32_ROTATIONS if fp32_rotations else 0)
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_server_add(self.handle, C.byref(problem.dims), C.byref(problem.model),
                                             C.byref(problem.map), int(precision), flags, X0.ctypes.data_as(_pd),
                                             C.byref(h)), "letkf_server_add")
        return Instance(self, h, problem, precision)

    def remove(self, inst: Instance):
        L.check(L.lib().letkf_server_remove(self.handle, inst.handle), "letkf_server_remove")
        inst.handle = None

    def submit(self, inst: Instance, y, frame_id: int, pred_out=None) -> int:
        """Queues one frame; returns the status (0, or -3 when the queue is full).
        y: host array (copied at once) or a float64 CUDA tensor (read in place by
        the batch's kernels; keep it unchanged until the frame is done)."""
        dev = isinstance(y, torch.Tensor) and y.is_cuda
        if dev:
            if y.dtype != torch.float64 or not y.is_contiguous() or y.numel() != inst.problem.p:
                raise ValueError("device y must be a contiguous float64 tensor of p values")
        else:
            y = _f64(y)
        out_ptr = None
        if pred_out is not None:
            if pred_out.dtype != np.float64 or pred_out.shape != (inst.problem.n_act,) or not pred_out.flags.c_contiguous:
                raise ValueError("pred_out must be a contiguous float64 array of n_act values")
            self._keep[int(frame_id)] = pred_out
            out_ptr = pred_out.ctypes.data_as(_pd)
        if dev:
            rc = L.lib().letkf_submit_frame_device(inst.handle, C.c_void_p(y.data_ptr()), int(frame_id), out_ptr,
                                                   self._cb, None)
        else:
            rc = L.lib().letkf_submit_frame(inst.handle, y.ctypes.data_as(_pd), int(frame_id), out_ptr, self._cb, None)
        if rc not in (L.OK, L.EAGAIN):
            self._keep.pop(int(frame_id), None)
            L.check(rc, "letkf_submit_frame")
        return rc

    def drain(self):
        L.check(L.lib().letkf_server_drain(self.handle), "letkf_server_drain")

    def set_window(self, window_us: int):
        L.check(L.lib().letkf_server_set_window(self.handle, int(window_us)), "letkf_server_set_window")

    def autotune(self, reps: int = 3) -> dict:
        """Per-class analysis launch shapes timed on the admitted instances
        (letkf_server_autotune, only while idle); returns {class index: choice}
        for the classes that have instances."""
        t = (L.Tuning * L.SERVER_CLASSES)()
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_server_autotune(self.handle, int(reps), t), "letkf_server_autotune")
        return {c: t[c].as_dict() for c in range(L.SERVER_CLASSES) if t[c].candidates > 0}

    def set_tuning(self, cls: int, grid: int, order: int = L.ORDER_COST):
        """Sets one class's analysis grid and its instances' domain order (idle only)."""
        t = L.Tuning(grid=int(grid), order=int(order))
        with torch.cuda.device(self.device):
            L.check(L.lib().letkf_server_set_tuning(self.handle, int(cls), C.byref(t)), "letkf_server_set_tuning")

    def stats(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        L.check(L.lib().letkf_server_stats(self.handle, C.byref(a), C.byref(b), C.byref(c)), "letkf_server_stats")
        return dict(frames=int(a.value), batches=int(b.value), batched_frames=int(c.value))

    def close(self):
        if getattr(self, "handle", None):
            L.lib().letkf_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
