"""Closed-loop single-conjugate AO around a filter: the paper's simulation
setting (Sec. 3), in which its controllers are compared by coherent energy.

* Truth: the case's frozen-flow screens, read at the actuator points (for the
  slopes) and at P x P points per valid subaperture (P = 10 in Sec. 3) for
  the residual phase.
* Deformable mirror: instantaneous, Gaussian influence functions whose value
  at the neighbouring actuator (the coupling) is 0.3, cut off beyond 2
  pitches.
* Wavefront sensor: y = D (phi - phi_dm) + noise at the actuator points (the
  case's D and slope noise).
* Two-frame delay: the command applied from frame k + 2 on is computed from
  the slopes of frame k.
* Pseudo-open-loop slopes: the filter sees y + D phi_dm (the mirror's known
  contribution added back), the slopes of the turbulence alone, and returns
  the means of phi_k (analysis) and phi_{k+1} (prediction); the command for
  frame k + 2 fits the mirror at the actuator points to the AR(2) extrapolation
  phi_{k+2|k} = a1 phi_{k+1|k} + a2 phi_{k|k}.
* Quality: coherent energy E = exp(-s2), s2 the piston-removed spatial
  variance of the residual phase over the fine points, averaged over the
  frames after the burn-in.

Reading: the paper does not give the influence function's shape, the fitting
rule or the extrapolation used against the delay; those above are this
module's.  It holds none of the filter's arithmetic: the filter is a callable
(the HIP library's plain path, or the oracle in the tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.spatial import cKDTree

from .configs import PITCH, Case

COUPLING = 0.3
CUTOFF = 2.0     # influence radius in pitches
DELAY = 2        # frames between a measurement and the command it produces
FINE = 10        # residual points per subaperture side


def fine_points(geom, per_side: int = FINE, pitch: float = PITCH) -> np.ndarray:
    """Metric (x, y) of per_side x per_side points in every valid subaperture
    (subaperture (r, c) spans actuator columns c..c+1 and rows r..r+1)."""
    u = (np.arange(per_side) + 0.5) / per_side
    gx, gy = np.meshgrid(u, u)
    rc = geom.sub_rc.astype(float)
    x = (rc[:, 1][:, None] + gx.ravel()[None, :]) * pitch
    y = (rc[:, 0][:, None] + gy.ravel()[None, :]) * pitch
    return np.stack([x.ravel(), y.ravel()], axis=1)


def influence_matrix(points_xy: np.ndarray, act_xy: np.ndarray, coupling: float = COUPLING,
                     pitch: float = PITCH, cutoff: float = CUTOFF) -> sp.csr_matrix:
    """F[i, j] = coupling^((d_ij / pitch)^2) for d_ij <= cutoff pitches."""
    tree_p, tree_a = cKDTree(points_xy), cKDTree(act_xy)
    dist = tree_p.sparse_distance_matrix(tree_a, cutoff * pitch * (1 + 1e-12), output_type="coo_matrix")
    d2 = (dist.data / pitch) ** 2
    return sp.coo_matrix((coupling ** d2, (dist.row, dist.col)), shape=(len(points_xy), len(act_xy))).tocsr()


class ClosedLoop:
    def __init__(self, case: Case, per_side: int = FINE):
        self.case = case
        geom = case.geom
        self.act_xy = geom.act_rc[:, ::-1].astype(float) * PITCH
        self.fine_xy = fine_points(geom, per_side)
        self.F_act = influence_matrix(self.act_xy, self.act_xy)
        self.F_fine = influence_matrix(self.fine_xy, self.act_xy)
        self._solve = spla.factorized(self.F_act.tocsc())
        self.D = sp.csr_matrix((case.D.val, case.D.col, case.D.rowptr), shape=case.D.shape)

    def fit(self, phi_act: np.ndarray) -> np.ndarray:
        """Commands whose mirror shape equals phi_act at the actuator points."""
        return self._solve(phi_act)

    def perfect_step(self):
        """A controller that knows the truth: it returns the true phi_k and
        phi_{k+1} at the actuator points, so that the command for frame k + 2
        fits a1 phi_{k+1} + a2 phi_k; its residual is the fitting and AR-model
        floor of this mirror (a bound for every filter)."""
        state = dict(k=0)

        def step(_y):
            k = state["k"]
            state["k"] += 1
            return self.case.truth.phase(k * 1e-3), self.case.truth.phase((k + 1) * 1e-3)
        return step

    def run(self, step, frames: int, burn_in: int) -> dict:
        """step(y_pol) -> (mean of phi_k, mean of phi_{k+1}) of the filter fed frame k."""
        case, n = self.case, self.case.n_act
        cmd = [np.zeros(n) for _ in range(frames + DELAY)]
        s2_cl, s2_ol = [], []
        for k in range(frames):
            t = k * 1e-3
            phi_act = case.truth.phase(t)
            phi_fine = case.truth.phase_at(self.fine_xy, t)
            dm_act = self.F_act @ cmd[k]
            res_fine = phi_fine - self.F_fine @ cmd[k]
            s2_cl.append(float(np.var(res_fine)))
            s2_ol.append(float(np.var(phi_fine)))
            noise = case.slopes(k) - self.D @ phi_act     # the case's slope noise of frame k
            y_res = self.D @ (phi_act - dm_act) + noise    # what the sensor measures in closed loop
            y_pol = y_res + self.D @ dm_act                # pseudo-open-loop slopes
            amean, pmean = step(y_pol)
            cmd[k + DELAY] = self.fit(case.a1 * pmean + case.a2 * amean)
        s2 = float(np.mean(s2_cl[burn_in:]))
        s2o = float(np.mean(s2_ol[burn_in:]))
        return dict(coherent_energy=float(np.exp(-s2)), residual_var=s2, open_loop_var=s2o,
                    open_loop_coherent_energy=float(np.exp(-s2o)), frames=frames, burn_in=burn_in,
                    commands=np.array(cmd[:frames + DELAY]), residual_series=np.array(s2_cl))
