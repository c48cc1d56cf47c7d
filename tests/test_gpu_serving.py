"""GPU serving: continuous batching across resident instances.

* A frame's result is the same alone and in the mix, where it shares a
  launch with frames of its class and runs beside batches of other classes
  (bit-identical: per-domain work has a fixed order and the merge uses no
  atomics).
* The server path equals the plain per-frame path.
* Instances are admitted against the HBM budget and re-admitted when
  memory frees up.
"""
import functools

import numpy as np
import pytest

from paper_1310_5954_amd import BF16, FP32, FP64, Filter, LetkfError, Problem, Server
from paper_1310_5954_amd import _lib as L
from workload.configs import build_case

pytestmark = pytest.mark.gpu

FRAMES = 8


@functools.lru_cache(maxsize=1)
def _mix_cases():
    """Seven classes (padded ensemble size x arithmetic variant) and, in the
    first class, two instances with different pupils and ensembles, so that
    some batches share launches and batches of other classes run beside them.
    The 100x100, m = 128 BF16 instance is the serving workload's largest: its
    workgroups fill a CU each, so while the other classes are resident its
    analysis runs on at most 3/4 of the CUs.  The 24x24 BF16 instance also
    runs with the opt-in FP32 rotations, a class of its own."""
    c16 = dict(build_case(2).cfg)
    c16.update(lenslets=16, seeds=(21, 22, 23))
    c24 = dict(build_case(2).cfg)
    c24.update(lenslets=24, seeds=(31, 32, 33), m=64)
    c12 = dict(build_case(1).cfg)
    c12.update(lenslets=12, seeds=(41, 42, 43), window=3, stride=3)
    c100 = dict(build_case(3).cfg)
    c100.update(lenslets=100, seeds=(51, 52, 53), frames=20)
    return [(build_case(1), FP64, {}), (build_case(c12), FP64, {}), (build_case(2), FP32, {}),
            (build_case(c16, m=20), FP64, {}), (build_case(c24), BF16, {}), (build_case(1, m=33), FP64, {}),
            (build_case(c100, m=128), BF16, {}), (build_case(c24), BF16, dict(fp32_rotations=True))]


def _run_server(cases, frames=FRAMES, drain_each=False, budget=1 << 31, graphs=False, tune=False, grid=None):
    srv = Server(budget, graphs=graphs)
    insts = [srv.add(Problem.from_case(c), c.X0, p, **kw) for c, p, kw in cases]
    if tune:
        choice = srv.autotune(reps=1)
        classes = {L_class(c.m, p, kw.get("fp32_rotations", False)) for c, p, kw in cases}
        assert set(choice) == classes, (choice, classes)
        assert all(1 <= t["grid"] and t["candidates"] >= 2 for t in choice.values()), choice
    if grid is not None:                 # persistent analysis with `grid` workgroups, map order
        for cls in range(L.SERVER_CLASSES):
            srv.set_tuning(cls, grid, order=L.ORDER_XCD if grid > 1 else L.ORDER_MAP)
        # the balanced order is for plain instances: a batch's placement depends on the batch
        with pytest.raises(LetkfError):
            srv.set_tuning(0, grid, order=L.ORDER_BALANCED)
    ys = [[c.slopes(k) for k in range(frames)] for c, _, _ in cases]
    preds = [[np.empty(c.n_act) for _ in range(frames)] for c, _, _ in cases]
    for k in range(frames):
        for i, inst in enumerate(insts):
            assert srv.submit(inst, ys[i][k], 1000 * i + k, preds[i][k]) == 0
        if drain_each:
            srv.drain()
    srv.drain()
    assert all(st == 0 for st, _ in srv.done.values())
    assert len(srv.done) == frames * len(cases)
    states = [inst.get_state() for inst in insts]
    stats = srv.stats()
    srv.close()
    return preds, states, stats


def L_class(m, precision, fp32_rotations=False):
    """Class index of an instance: arithmetic variant x 4 + padded-size index
    (variant: the precision, or 3 for BF16 with FP32 rotations)."""
    pm = 16
    while pm < m:
        pm *= 2
    variant = 3 if fp32_rotations else precision
    return variant * 4 + {16: 0, 32: 1, 64: 2, 128: 3}[pm]


@pytest.mark.parametrize("graphs,tune,grid", [(True, False, None), (True, True, None), (False, False, 2),
                                              (True, False, 5)])
def test_graphs_tuning_and_grid_leave_mix_results_unchanged(graphs, tune, grid):
    """Replayed batch graphs (LETKF_SERVER_GRAPHS), autotuned launch shapes,
    and a persistent analysis grid far below the domain count (the
    workgroups claim the remaining domains through the work counter) give
    the mix the same predictions and states, bit for bit, as the default
    one-by-one launches."""
    cases = _mix_cases()
    ref_preds, ref_states, _ = _run_server(cases)
    preds, states, _ = _run_server(cases, graphs=graphs, tune=tune, grid=grid)
    for i in range(len(cases)):
        for k in range(FRAMES):
            assert np.array_equal(ref_preds[i][k], preds[i][k]), (i, k)
        assert np.array_equal(ref_states[i][0], states[i][0]) and ref_states[i][1] == states[i][1], i


def test_alone_vs_in_the_mix_bit_identical():
    cases = _mix_cases()
    mixed_preds, mixed_states, stats = _run_server(cases)
    assert stats["batched_frames"] > stats["batches"], stats    # some frames really shared launches
    for i, cp in enumerate(cases):
        alone_preds, alone_states, _ = _run_server([cp], drain_each=True)
        for k in range(FRAMES):
            assert np.array_equal(alone_preds[0][k], mixed_preds[i][k]), (i, k)
        assert np.array_equal(alone_states[0][0], mixed_states[i][0]), i
        assert alone_states[0][1] == mixed_states[i][1] == FRAMES


def test_server_pistons_equal_plain_pistons():
    """A server instance with differential-piston removal gives the same
    predictions as the plain path with it."""
    cfg = dict(build_case(2).cfg)
    cfg.update(lenslets=16)
    case = build_case(cfg)
    srv = Server(1 << 30)
    inst = srv.add(Problem.from_case(case), case.X0, FP64, pistons=True)
    preds = [np.empty(case.n_act) for _ in range(4)]
    for k in range(4):
        assert srv.submit(inst, case.slopes(k), k, preds[k]) == 0
    srv.drain()
    srv.close()
    f = Filter(Problem.from_case(case), case.X0, precision=FP64, pistons=True)
    for k in range(4):
        assert np.array_equal(f.step(case.slopes(k), pred=True), preds[k]), k


def test_server_equals_plain_path():
    case = build_case(1)
    preds, states, _ = _run_server([(case, FP64, {})], drain_each=True)
    f = Filter(Problem.from_case(case), case.X0, precision=FP64)
    for k in range(FRAMES):
        p = f.step(case.slopes(k), pred=True)
        assert np.array_equal(p, preds[0][k]), k
    X, fr = f.get_state()
    assert np.array_equal(X, states[0][0]) and fr == FRAMES


def test_admission_by_hbm_budget():
    case = build_case(3)
    pr = Problem.from_case(case)
    ws = pr.workspace_size(FP64)
    assert ws > 16 << 20
    server_tables = L.lib().letkf_server_reserved_bytes()   # staging and tables of the server itself
    srv = Server(server_tables + int(2.5 * ws))
    a = srv.add(pr, case.X0, FP64)
    b = srv.add(pr, case.X0, FP64)
    with pytest.raises(LetkfError) as ei:
        srv.add(pr, case.X0, FP64)    # half a workspace short
    assert ei.value.status == -2
    y = case.slopes(0)
    out = np.empty(case.n_act)
    srv.submit(a, y, 1, out)
    srv.drain()
    srv.remove(a)                      # memory frees up ...
    c = srv.add(pr, case.X0, FP64)    # ... and the waiting instance is admitted
    srv.submit(c, y, 2, np.empty(case.n_act))
    srv.submit(b, y, 3, np.empty(case.n_act))
    srv.drain()
    assert srv.done[2][0] == 0 and srv.done[3][0] == 0
    srv.close()


def test_plain_calls_refused_on_server_instances():
    case = build_case(1)
    srv = Server(1 << 28)
    inst = srv.add(Problem.from_case(case), case.X0, FP64)
    from paper_1310_5954_amd import _lib as L
    import ctypes as C
    rc = L.lib().letkf_forecast(inst.handle, None)
    assert rc == L.ESTATE
    rc = L.lib().letkf_destroy(inst.handle)
    assert rc == L.ESTATE
    srv.close()


def test_device_slopes_equal_host_slopes():
    """letkf_submit_frame_device reads the caller's device buffer in place and
    gives the same bits as host submission."""
    import torch
    case = build_case(1)
    host_preds, host_states, _ = _run_server([(case, FP64, {})], drain_each=True)
    srv = Server(1 << 28)
    inst = srv.add(Problem.from_case(case), case.X0, FP64)
    ys = [torch.tensor(case.slopes(k), dtype=torch.float64, device="cuda:0") for k in range(FRAMES)]
    preds = [np.empty(case.n_act) for _ in range(FRAMES)]
    for k in range(FRAMES):
        assert srv.submit(inst, ys[k], k, preds[k]) == 0
    srv.drain()
    for k in range(FRAMES):
        assert np.array_equal(preds[k], host_preds[0][k]), k
    X, fr = inst.get_state()
    assert np.array_equal(X, host_states[0][0]) and fr == FRAMES
    srv.close()


def test_callback_may_submit_next_frame():
    """Closed loop driven from the completion callback (the serving bench's pattern)."""
    import threading
    case = build_case(1)
    done = threading.Event()
    order = []
    srv = None

    def on_done(fid, status, t):
        order.append(fid)
        if fid + 1 < FRAMES:
            srv.submit(inst, case.slopes(fid + 1), fid + 1, np.empty(case.n_act))
        else:
            done.set()

    srv = Server(1 << 28, on_done=on_done)
    inst = srv.add(Problem.from_case(case), case.X0, FP64)
    srv.submit(inst, case.slopes(0), 0, np.empty(case.n_act))
    assert done.wait(60)
    srv.drain()
    assert order == list(range(FRAMES))
    srv.close()


def test_nonfinite_device_slopes_refused_and_state_kept():
    """Device slopes are checked by the slope kernel: a frame with a NaN is
    reported with LETKF_ENUMERIC, leaves its instance's ensemble and frame
    counter as they were, and the frames after it run as if it had never
    been submitted (equal, bit for bit, to a run without it)."""
    import torch
    case = build_case(1)
    ref_preds, ref_states, _ = _run_server([(case, FP64, {})], frames=3, drain_each=True)
    srv = Server(1 << 28)
    inst = srv.add(Problem.from_case(case), case.X0, FP64)
    good = [torch.tensor(case.slopes(k), dtype=torch.float64, device="cuda:0") for k in range(3)]
    bad = good[1].clone()
    bad[7] = float("nan")
    preds = [np.empty(case.n_act) for _ in range(4)]
    seq = [(good[0], 0), (bad, 1), (good[1], 2), (good[2], 3)]
    for y, fid in seq:
        assert srv.submit(inst, y, fid, preds[fid]) == 0
        srv.drain()
        if fid == 1:
            X, fr = inst.get_state()
            assert fr == 1                              # the refused frame advanced nothing
    assert srv.done[1][0] == L.ENUMERIC
    assert all(srv.done[f][0] == 0 for f in (0, 2, 3))
    for k, fid in ((0, 0), (1, 2), (2, 3)):
        assert np.array_equal(preds[fid], ref_preds[0][k]), (k, fid)
    X, fr = inst.get_state()
    assert fr == 3 and np.array_equal(X, ref_states[0][0])
    srv.close()


def test_autotune_runs_without_blocking_submitters():
    """letkf_server_autotune times its launches without holding the server
    lock: a frame submitted meanwhile is queued at once (the call returns in
    well under the tuning time) and launched after the tuning, with the same
    result as without tuning."""
    import threading
    import time
    case = build_case(3)
    ref_preds, _, _ = _run_server([(case, BF16, {})], frames=1)
    srv = Server(1 << 30)
    inst = srv.add(Problem.from_case(case), case.X0, BF16)
    t_tune = {}

    def tune():
        t0 = time.perf_counter()
        srv.autotune(reps=30)
        t_tune["s"] = time.perf_counter() - t0

    th = threading.Thread(target=tune)
    th.start()
    time.sleep(0.05)                 # the tuning is under way
    pred = np.empty(case.n_act)
    t0 = time.perf_counter()
    rc = srv.submit(inst, case.slopes(0), 0, pred)
    t_submit = time.perf_counter() - t0
    during = th.is_alive()           # the submission returned while the tuning ran
    th.join()
    srv.drain()
    assert rc == 0 and srv.done[0][0] == 0
    print(f"autotune {t_tune['s']:.3f} s, submit during it {1e3 * t_submit:.2f} ms", flush=True)
    assert during and t_submit < 0.1 and t_submit < t_tune["s"] / 4, (during, t_submit, t_tune)
    assert np.array_equal(pred, ref_preds[0][0])
    srv.close()
