"""The closed loop of Sec. 3 with the HIP library's plain FP64 path as the
filter equals the same loop with the oracle: the mirror commands (which
depend on the filter's analysis and prediction means every frame) and the
residual series agree to 1e-9 over 30 frames."""
import numpy as np
import pytest

from paper_1310_5954_amd import FP64, Filter, Problem
from test_closed_loop import _case, _oracle_step
from workload.closed_loop import ClosedLoop

pytestmark = pytest.mark.gpu


def test_closed_loop_gpu_filter_equals_oracle_filter():
    case = _case()
    cl = ClosedLoop(case)
    f = Filter(Problem.from_case(case), case.X0, precision=FP64)

    def gpu_step(y):
        f.step(y, pred=False)
        return f.last_means()
    g = cl.run(gpu_step, 30, 10)
    f.close()
    step, _ = _oracle_step(case)
    o = cl.run(step, 30, 10)
    cg, co = g["commands"], o["commands"]
    err = np.linalg.norm(cg - co) / np.linalg.norm(co)
    rs = np.max(np.abs(g["residual_series"] - o["residual_series"]) / o["residual_series"])
    print(f"[closed loop] commands rel err {err:.1e}, residual series rel err {rs:.1e}, "
          f"residual var {g['residual_var']:.3f} (open loop {g['open_loop_var']:.1f})", flush=True)
    assert err < 1e-9 and rs < 1e-9
