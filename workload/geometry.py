"""Shack-Hartmann / Fried geometry, the WFS matrix D and local-domain maps.

Seeded input generator shared by the oracle, the tests and the benchmark.  It
holds none of the filter's arithmetic: it only builds the *inputs* the
local ETKF is defined on (paper Sec. 2.1 state-space statement, Sec. 2.3
domain decomposition, Sec. 3 SH-WFS model).

Conventions
-----------
* An N x N lenslet grid of pitch d; subaperture (a, b) (row a, column b) has
  its four corners on the (N+1) x (N+1) actuator grid (Fried geometry, Sec. 2.3
  and the Fig. 1 caption).
* Pupil: a subaperture is valid when its illuminated fraction is at least
  ``threshold`` (Sec. 3: "transmission factor equal to 0.5"); the fraction is
  measured on a ``samples`` x ``samples`` grid of points.  An actuator is valid
  when it is a corner of a valid subaperture (Sec. 3: 241 valid actuators at
  16x16, 877 at 32x32).
* Valid subapertures and actuators are numbered in row-major grid order.
* D (Sec. 3, "difference of the phase at the edges of the subapertures"):
  for a subaperture with corner phases p00=(a,b), p01=(a,b+1), p10=(a+1,b),
  p11=(a+1,b+1)  (first index = row = y, second = column = x)
      s_x = ((p01 + p11) - (p00 + p10)) / 2
      s_y = ((p10 + p11) - (p00 + p01)) / 2
  in radians per pitch.  The slope vector is all s_x (subaperture order), then
  all s_y, so p = 2 * n_sub.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Geometry:
    n_lenslets: int               # N (lenslets across)
    shape: str                    # "circular" or "square"
    sub_mask: np.ndarray          # (N, N) bool
    act_mask: np.ndarray          # (N+1, N+1) bool
    sub_index: np.ndarray         # (N, N) int32, -1 where invalid
    act_index: np.ndarray         # (N+1, N+1) int32, -1 where invalid
    sub_rc: np.ndarray            # (n_sub, 2) int32 grid (row, col) of each subaperture
    act_rc: np.ndarray            # (n_act, 2) int32 grid (row, col) of each actuator

    @property
    def n_sub(self) -> int:
        return int(self.sub_rc.shape[0])

    @property
    def n_act(self) -> int:
        return int(self.act_rc.shape[0])

    @property
    def n(self) -> int:  # state dimension: two time instants per actuator
        return 2 * self.n_act

    @property
    def p(self) -> int:  # slope dimension: x and y per subaperture
        return 2 * self.n_sub


def illuminated_fraction(n_lenslets: int, samples: int = 20) -> np.ndarray:
    """Fraction of each subaperture inside the circle of diameter N pitches."""
    N = n_lenslets
    r = N / 2.0
    q = (np.arange(samples) + 0.5) / samples
    frac = np.zeros((N, N))
    for a in range(N):
        y = a + q[:, None] - r
        for b in range(N):
            x = b + q[None, :] - r
            frac[a, b] = np.mean(x * x + y * y <= r * r)
    return frac


def build_geometry(n_lenslets: int, shape: str = "circular", threshold: float = 0.5,
                   samples: int = 20) -> Geometry:
    N = int(n_lenslets)
    if N < 1:
        raise ValueError("need at least one lenslet")
    if shape == "square":
        sub_mask = np.ones((N, N), dtype=bool)
    elif shape == "circular":
        sub_mask = illuminated_fraction(N, samples) >= threshold
    else:
        raise ValueError(f"unknown pupil shape {shape!r}")
    act_mask = np.zeros((N + 1, N + 1), dtype=bool)
    for da in (0, 1):
        for db in (0, 1):
            act_mask[da:da + N, db:db + N] |= sub_mask
    sub_index = np.full((N, N), -1, dtype=np.int32)
    act_index = np.full((N + 1, N + 1), -1, dtype=np.int32)
    sub_rc = np.argwhere(sub_mask).astype(np.int32)
    act_rc = np.argwhere(act_mask).astype(np.int32)
    sub_index[sub_rc[:, 0], sub_rc[:, 1]] = np.arange(len(sub_rc), dtype=np.int32)
    act_index[act_rc[:, 0], act_rc[:, 1]] = np.arange(len(act_rc), dtype=np.int32)
    return Geometry(N, shape, sub_mask, act_mask, sub_index, act_index, sub_rc, act_rc)


@dataclass
class CSR:
    rowptr: np.ndarray  # int32 (rows+1)
    col: np.ndarray     # int32 (nnz)
    val: np.ndarray     # float64 (nnz)
    shape: tuple

    def to_dense(self) -> np.ndarray:
        out = np.zeros(self.shape)
        for r in range(self.shape[0]):
            for k in range(self.rowptr[r], self.rowptr[r + 1]):
                out[r, self.col[k]] += self.val[k]
        return out


def fried_slope_matrix(geom: Geometry) -> CSR:
    """D as CSR (p x n_act), four nonzeros per row, Sec. 3 WFS model."""
    ns = geom.n_sub
    rows_col = np.zeros((2 * ns, 4), dtype=np.int32)
    rows_val = np.zeros((2 * ns, 4))
    ai = geom.act_index
    for s, (a, b) in enumerate(geom.sub_rc):
        p00, p01 = ai[a, b], ai[a, b + 1]
        p10, p11 = ai[a + 1, b], ai[a + 1, b + 1]
        rows_col[s] = (p00, p01, p10, p11)
        rows_val[s] = (-0.5, 0.5, -0.5, 0.5)           # x: right column minus left column
        rows_col[ns + s] = (p00, p01, p10, p11)
        rows_val[ns + s] = (-0.5, -0.5, 0.5, 0.5)      # y: bottom row minus top row
    order = np.argsort(rows_col, axis=1, kind="stable")
    rows_col = np.take_along_axis(rows_col, order, axis=1)
    rows_val = np.take_along_axis(rows_val, order, axis=1)
    rowptr = np.arange(0, 4 * 2 * ns + 1, 4, dtype=np.int32)
    return CSR(rowptr, rows_col.reshape(-1).copy(), rows_val.reshape(-1).copy(),
               (2 * ns, geom.n_act))


# --------------------------------------------------------------------------
# Local domains (Sec. 2.3): estimation domains partition (or cover) the
# actuators; each has an observation region of surrounding subapertures.
# --------------------------------------------------------------------------

def gaspari_cohn(z: np.ndarray) -> np.ndarray:
    """Gaspari & Cohn (1999, eq. 4.10) compactly supported 5th-order taper."""
    z = np.abs(np.asarray(z, dtype=float))
    out = np.zeros_like(z)
    a = z <= 1.0
    b = (z > 1.0) & (z < 2.0)
    za = z[a]
    out[a] = -0.25 * za**5 + 0.5 * za**4 + 0.625 * za**3 - (5.0 / 3.0) * za**2 + 1.0
    zb = z[b]
    out[b] = (zb**5 / 12.0 - 0.5 * zb**4 + 0.625 * zb**3 + (5.0 / 3.0) * zb**2
              - 5.0 * zb + 4.0 - 2.0 / (3.0 * zb))
    return out


@dataclass
class DomainMap:
    est_ptr: np.ndarray    # int32 (L+1)
    est_act: np.ndarray    # int32  actuator indices per domain
    est_w: np.ndarray      # float64 merge weight of each (domain, actuator) entry
    obs_ptr: np.ndarray    # int32 (L+1)
    obs_sub: np.ndarray    # int32  subaperture indices per domain (both slopes used)
    obs_taper: np.ndarray  # float64 taper in [0, 1] applied to R^-1
    info: dict = field(default_factory=dict)

    @property
    def n_domains(self) -> int:
        return int(len(self.est_ptr) - 1)

    def est(self, l):
        return self.est_act[self.est_ptr[l]:self.est_ptr[l + 1]]

    def obs(self, l):
        return self.obs_sub[self.obs_ptr[l]:self.obs_ptr[l + 1]]

    def weights(self, l):
        return self.est_w[self.est_ptr[l]:self.est_ptr[l + 1]]

    def taper(self, l):
        return self.obs_taper[self.obs_ptr[l]:self.obs_ptr[l + 1]]

    def stats(self) -> dict:
        e = np.diff(self.est_ptr)
        s = np.diff(self.obs_ptr)
        return dict(n_domains=self.n_domains, e_min=int(e.min()), e_max=int(e.max()),
                    n_max=int(2 * e.max()), p_max=int(2 * s.max()),
                    sum_n=int(2 * e.sum()), sum_p=int(2 * s.sum()))


def _finish_map(geom: Geometry, domains: list, halo: int, taper: bool) -> DomainMap:
    """domains: list of (act_ids sorted, box=(i0,i1,j0,j1) in actuator rows/cols)."""
    count = np.zeros(geom.n_act, dtype=np.int64)
    for acts, _ in domains:
        count[acts] += 1
    if np.any(count == 0):
        raise ValueError("domain map leaves actuators uncovered")
    est_ptr, est_act, est_w = [0], [], []
    obs_ptr, obs_sub, obs_taper = [0], [], []
    c = (halo + 0.5) / 2.0  # Gaspari-Cohn half-support: support 2c = halo + 1/2 pitch
    N = geom.n_lenslets
    for acts, (i0, i1, j0, j1) in domains:
        est_act.extend(acts.tolist())
        est_w.extend((1.0 / count[acts]).tolist())
        est_ptr.append(len(est_act))
        a0, a1 = max(i0 - halo, 0), min(i1 + halo - 1, N - 1)
        b0, b1 = max(j0 - halo, 0), min(j1 + halo - 1, N - 1)
        subs = []
        for a in range(a0, a1 + 1):
            for b in range(b0, b1 + 1):
                s = geom.sub_index[a, b]
                if s >= 0:
                    subs.append(int(s))
        subs = np.array(sorted(subs), dtype=np.int64)
        if taper and len(subs):
            rc = geom.sub_rc[subs].astype(float) + 0.5
            dy = np.maximum(np.maximum(i0 - rc[:, 0], rc[:, 0] - i1), 0.0)
            dx = np.maximum(np.maximum(j0 - rc[:, 1], rc[:, 1] - j1), 0.0)
            t = gaspari_cohn(np.hypot(dx, dy) / c)
        else:
            t = np.ones(len(subs))
        obs_sub.extend(subs.tolist())
        obs_taper.extend(t.tolist())
        obs_ptr.append(len(obs_sub))
    return DomainMap(np.array(est_ptr, np.int32), np.array(est_act, np.int32),
                     np.array(est_w, np.float64), np.array(obs_ptr, np.int32),
                     np.array(obs_sub, np.int32), np.array(obs_taper, np.float64),
                     info=dict(halo=halo, taper=taper))


def window_domains(geom: Geometry, window: int, stride: int, halo: int, taper: bool = False,
                   min_actuators: int = 0, shift: int = 0) -> DomainMap:
    """Square actuator windows of side ``window`` every ``stride`` actuators,
    centred on the actuator grid; observation region = subaperture rows
    [i0-halo, i1+halo-1] x columns [j0-halo, j1+halo-1] of each window
    [i0, i1] x [j0, j1].  Windows with fewer than ``min_actuators`` valid
    actuators are dropped when other windows cover all their actuators, and
    otherwise merged into the kept window sharing the most actuators (the
    nearest one when none is shared).  ``shift`` (0 < shift < stride) moves
    the window grid by that many actuators along both axes, with one more
    window per axis so that the edges stay covered: a staggered partition."""
    side = geom.n_lenslets + 1
    nw = max(1, math.ceil(max(side - window, 0) / stride) + 1)
    span = (nw - 1) * stride + window
    off = (side - span) // 2
    if shift:
        off += shift - stride
        nw += 1
    raw = []
    for wi in range(nw):
        for wj in range(nw):
            i0, j0 = off + wi * stride, off + wj * stride
            i1, j1 = i0 + window - 1, j0 + window - 1
            sub = geom.act_index[max(i0, 0):min(i1, side - 1) + 1, max(j0, 0):min(j1, side - 1) + 1]
            acts = np.sort(sub[sub >= 0]).astype(np.int64)
            if len(acts):
                raw.append([acts, (i0, i1, j0, j1)])
    if min_actuators > 0:
        big = [d for d in raw if len(d[0]) >= min_actuators]
        small = [d for d in raw if len(d[0]) < min_actuators]
        covered = np.zeros(geom.n_act, dtype=bool)
        for acts, _ in big:
            covered[acts] = True
        for acts, box in small:
            if covered[acts].all():
                continue
            shared = [len(np.intersect1d(acts, b[0])) for b in big]
            if max(shared) > 0:
                k = int(np.argmax(shared))
            else:
                cy, cx = (box[0] + box[1]) / 2, (box[2] + box[3]) / 2
                dist = [math.hypot((b[1][0] + b[1][1]) / 2 - cy, (b[1][2] + b[1][3]) / 2 - cx)
                        for b in big]
                k = int(np.argmin(dist))
            b_acts, b_box = big[k]
            big[k] = [np.union1d(b_acts, acts),
                      (min(b_box[0], box[0]), max(b_box[1], box[1]),
                       min(b_box[2], box[2]), max(b_box[3], box[3]))]
            covered[acts] = True
        raw = big
    return _finish_map(geom, [(d[0], d[1]) for d in raw], halo, taper)


def block_partition(geom: Geometry, block: int, offset: int, halo: int, taper: bool = False,
                    min_actuators: int = 0) -> DomainMap:
    """Non-overlapping square blocks of ``block`` actuators, grid shifted by
    ``offset`` (the Sec. 3.2 complexity examples)."""
    side = geom.n_lenslets + 1
    starts = list(range(-offset, side, block))
    raw = []
    for i0 in starts:
        for j0 in starts:
            i1, j1 = i0 + block - 1, j0 + block - 1
            sub = geom.act_index[max(i0, 0):min(i1, side - 1) + 1, max(j0, 0):min(j1, side - 1) + 1]
            acts = np.sort(sub[sub >= 0]).astype(np.int64)
            if len(acts):
                raw.append([acts, (i0, i1, j0, j1)])
    if min_actuators > 0:
        big = [d for d in raw if len(d[0]) >= min_actuators]
        for acts, box in [d for d in raw if len(d[0]) < min_actuators]:
            cy, cx = (box[0] + box[1]) / 2, (box[2] + box[3]) / 2
            # merge into the adjacent kept block whose box touches this one, nearest centre first
            dist = [math.hypot((b[1][0] + b[1][1]) / 2 - cy, (b[1][2] + b[1][3]) / 2 - cx) for b in big]
            k = int(np.argmin(dist))
            b_acts, b_box = big[k]
            big[k] = [np.union1d(b_acts, acts),
                      (min(b_box[0], box[0]), max(b_box[1], box[1]),
                       min(b_box[2], box[2]), max(b_box[3], box[3]))]
        raw = big
    return _finish_map(geom, [(d[0], d[1]) for d in raw], halo, taper)


def global_domain(geom: Geometry) -> DomainMap:
    """One domain holding every actuator and every subaperture (global ETKF)."""
    side = geom.n_lenslets + 1
    acts = np.arange(geom.n_act, dtype=np.int64)
    return _finish_map(geom, [(acts, (0, side - 1, 0, side - 1))], halo=side, taper=False)


def combine_maps(maps: list) -> DomainMap:
    """One map holding the domains of every map in ``maps``, with each map's
    merge weights divided by ``len(maps)``: the analysis on it is the equal-
    weight average of the analyses on the separate maps (several partitions
    of the pupil run in the same frame, Sec. 5)."""
    k = float(len(maps))
    est_ptr, obs_ptr = [0], [0]
    est_act, est_w, obs_sub, obs_taper = [], [], [], []
    for dm in maps:
        for l in range(dm.n_domains):
            est_act.append(dm.est(l)); est_w.append(dm.weights(l) / k)
            obs_sub.append(dm.obs(l)); obs_taper.append(dm.taper(l))
            est_ptr.append(est_ptr[-1] + len(dm.est(l)))
            obs_ptr.append(obs_ptr[-1] + len(dm.obs(l)))
    return DomainMap(np.array(est_ptr, np.int32), np.concatenate(est_act).astype(np.int32),
                     np.concatenate(est_w), np.array(obs_ptr, np.int32),
                     np.concatenate(obs_sub).astype(np.int32), np.concatenate(obs_taper),
                     info=dict(partitions=len(maps), parts=[dm.info for dm in maps]))
