"""The closed-loop harness around the filter (Sec. 3 setting), CPU checks.

Pins: the mirror's influence functions (coupling 0.3 at the neighbour, 1 on
the actuator), the command fit reproducing a mirror shape exactly, no
correction = open loop, the pseudo-open-loop slopes equal the turbulence's own
slopes, and the oracle filter in the loop lowering the residual well below the
open loop and staying above the truth-fed controller's floor."""
import numpy as np
import scipy.sparse as sp

import oracle
from workload.closed_loop import ClosedLoop, fine_points
from workload.configs import build_case


def _case():
    cfg = dict(build_case(2).cfg)
    cfg.update(lenslets=16)
    return build_case(cfg)


def _oracle_step(case):
    D = sp.csr_matrix((case.D.val, case.D.col, case.D.rowptr), shape=case.D.shape)
    st = dict(X=case.X0.copy(), k=0, ys=[])

    def step(y):
        st["ys"].append(y.copy())
        Xa, Xf = oracle.frame_step(st["X"], y, D, case.dmap, case.r_inv, case.a1, case.a2, case.sigma_v,
                                   case.philox_seed, st["k"])
        st["X"], st["k"] = Xf, st["k"] + 1
        return Xa[:case.n_act].mean(axis=1), Xf[:case.n_act].mean(axis=1)
    return step, st


def test_influence_functions_and_fit():
    case = _case()
    cl = ClosedLoop(case)
    assert np.allclose(cl.F_act.diagonal(), 1.0)
    ar = case.geom.act_rc
    # an interior actuator: its 4 neighbours at one pitch read 0.3, the diagonal ones 0.09
    i = next(i for i in range(case.n_act) if sum(((ar == ar[i] + d).all(axis=1)).any()
                                                 for d in ((0, 1), (1, 0), (0, -1), (-1, 0), (1, 1))) == 5)
    row = cl.F_act[i].toarray().ravel()
    for d, v in (((0, 1), 0.3), ((1, 0), 0.3), ((1, 1), 0.09)):
        j = int(np.where((ar == ar[i] + np.array(d)).all(axis=1))[0][0])
        assert abs(row[j] - v) < 1e-15
    c = np.random.default_rng(1).standard_normal(case.n_act)
    assert np.max(np.abs(cl.fit(cl.F_act @ c) - c)) < 1e-12
    assert fine_points(case.geom).shape == (100 * case.n_sub, 2)


def test_no_correction_is_open_loop_and_slopes_are_pseudo_open_loop():
    case = _case()
    cl = ClosedLoop(case)
    seen = []

    def step(y):
        seen.append(y.copy())
        return np.zeros(case.n_act), np.zeros(case.n_act)
    r = cl.run(step, 6, 2)
    assert r["residual_var"] == r["open_loop_var"]
    for k, y in enumerate(seen):
        assert np.allclose(y, case.slopes(k), rtol=0, atol=1e-12)


def test_oracle_in_the_loop_beats_open_loop_and_respects_the_floor():
    case = _case()
    cl = ClosedLoop(case)
    step, st = _oracle_step(case)
    r = cl.run(step, 40, 15)
    floor = cl.run(cl.perfect_step(), 40, 15)
    assert r["residual_var"] < 0.2 * r["open_loop_var"], r["residual_var"]
    assert floor["residual_var"] < r["residual_var"]
    # pseudo-open-loop slopes: the filter saw the turbulence's own slopes whatever the mirror did
    for k, y in enumerate(st["ys"]):
        assert np.allclose(y, case.slopes(k), rtol=0, atol=1e-10)
