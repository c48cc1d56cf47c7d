"""letkf_step_noalloc: the plain frame with its scratch in the library's
static device array (no allocation of any kind), against letkf_step on a twin
instance: the same predictions and states, bit for bit, over two calls in a
row on one GPU, the second on a smaller instance (the array keeps the first
call's contents)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1310_5954_amd import BF16, FP64, Filter, Problem
from paper_1310_5954_amd import _lib as L
from workload.configs import build_case

pytestmark = pytest.mark.gpu


def _noalloc_frames(case, precision, frames):
    pr = Problem.from_case(case)
    ref = Filter(pr, case.X0, precision=precision)
    f = Filter(pr, case.X0, precision=precision)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for k in range(frames):
        y = case.slopes(k)
        want = ref.step(y, pred=True)
        y_dev = torch.tensor(y, dtype=torch.float64, device="cuda:0")
        pred_dev = torch.full((case.n_act,), float("nan"), dtype=torch.float64, device="cuda:0")
        rc = L.lib().letkf_step_noalloc(f.handle, C.c_void_p(y_dev.data_ptr()), C.c_void_p(pred_dev.data_ptr()),
                                        stream)
        assert rc == L.OK, L.lib().letkf_last_error()
        torch.cuda.synchronize()
        got = pred_dev.cpu().numpy()
        assert np.array_equal(got, want), (case.cfg["name"], precision, k, np.abs(got - want).max())
    Xr, fr = ref.get_state()
    Xf, ff = f.get_state()
    assert fr == ff == frames and np.array_equal(Xr, Xf)
    ref.close()
    f.close()


def test_noalloc_step_equals_letkf_step_two_calls_then_smaller():
    """84x84, m = 64 (375 domains, FP64 scratch ~25 MB of the 32 MiB), then the
    15x15, m = 16 instance, then the 84x84 instance on the BF16 path."""
    _noalloc_frames(build_case(3), FP64, 2)
    _noalloc_frames(build_case(1), FP64, 2)
    _noalloc_frames(build_case(3), BF16, 2)


def test_noalloc_step_refuses_frames_beyond_the_static_maximum():
    """128x128, m = 128 in FP64 needs ~140 MB of frame scratch: refused before
    any device work, with the sizes in the message."""
    case = build_case(5)
    f = Filter(Problem.from_case(case), case.X0, precision=FP64)
    y_dev = torch.zeros(case.n_sub * 2, dtype=torch.float64, device="cuda:0")
    pred_dev = torch.zeros(case.n_act, dtype=torch.float64, device="cuda:0")
    X0, f0 = f.get_state()
    rc = L.lib().letkf_step_noalloc(f.handle, C.c_void_p(y_dev.data_ptr()), C.c_void_p(pred_dev.data_ptr()), None)
    assert rc == L.EINVAL
    assert b"static maximum" in L.lib().letkf_last_error()
    X1, f1 = f.get_state()
    assert f1 == f0 and np.array_equal(X0, X1)
    f.close()
