"""The five synthetic workloads and a builder for all inputs of one of them.

Every array is seeded.  The cases stand in for the paper's Matlab AO
simulation (Sec. 3: von Karman layers, Taylor frozen flow, SH WFS in Fried
geometry, 500 Hz-class frame loop) at the sizes this library targets:

  cfg1  15x15 square SH, 16x16 actuators, m=16, 16 disjoint 4x4 domains, halo 1, FP64
  cfg2  40x40 circular,  m=32, 5x5 windows stride 3, halo 2, Gaspari-Cohn taper, FP32
  cfg3  84x84 circular,  m=64, 6x6 windows stride 4, halo 2, taper, small windows merged, BF16
  cfg4  six instances (20, 40, 60, 84, 84, 100 lenslets) for the serving loop
  cfg5  128x128 circular, m=128, two layers, BF16/FP32 vs FP64

Slopes are pseudo-open-loop measurements y_k = D phi_k + N(0, sigma^2 I).
The AR(2) model is diagonal with a1 = 1.6, a2 = -0.64 (a double pole at
0.8); the model-noise std sigma_v is set so that the AR(2) stationary
variance sigma_v^2 (1 - a2) / ((1 + a2)((1 - a2)^2 - a1^2)) equals the
piston-removed per-actuator variance of the truth at t = 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import (CSR, DomainMap, Geometry, build_geometry, combine_maps, fried_slope_matrix,
                       global_domain, window_domains)
from .turbulence import FrozenFlow, independent_screens_at

PITCH = 0.5      # subaperture pitch d [m]
DT = 1.0e-3      # frame period [s]
SIGMA = 0.1      # slope noise std [rad]
A1, A2 = 1.6, -0.64

PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
PREC_NAMES = {PREC_FP64: "fp64", PREC_FP32: "fp32", PREC_BF16: "bf16"}


def ar2_stationary_gain(a1: float, a2: float) -> float:
    return (1 - a2) / ((1 + a2) * ((1 - a2) ** 2 - a1 ** 2))


CONFIGS = {
    1: dict(name="cfg1", lenslets=15, shape="square", m=16, window=4, stride=4, halo=1, taper=False,
            min_actuators=0, precision=PREC_FP64, r0=0.15, L0=25.0, layers=[dict(weight=1.0, speed=10.0)],
            frames=200, seeds=(1310, 5954, 1), philox_seed=0x13105954_0001),
    2: dict(name="cfg2", lenslets=40, shape="circular", m=32, window=5, stride=3, halo=2, taper=True,
            min_actuators=0, precision=PREC_FP32, r0=0.12, L0=30.0, layers=[dict(weight=1.0, speed=10.0)],
            frames=500, seeds=(1311, 5955, 2), philox_seed=0x13105954_0002),
    3: dict(name="cfg3", lenslets=84, shape="circular", m=64, window=6, stride=4, halo=2, taper=True,
            min_actuators=8, precision=PREC_BF16, r0=0.12, L0=30.0,
            layers=[dict(weight=1.0, speed=("ramp", 10.0, 25.0, 1.0))],
            frames=1000, seeds=(1312, 5956, 3), philox_seed=0x13105954_0003),
    5: dict(name="cfg5", lenslets=128, shape="circular", m=128, window=6, stride=4, halo=2, taper=True,
            min_actuators=8, precision=PREC_BF16, r0=0.10, L0=30.0,
            layers=[dict(weight=0.6, speed=10.0, angle_deg=0.0), dict(weight=0.4, speed=20.0, angle_deg=90.0)],
            frames=2000, seeds=(1314, 5958, 5), philox_seed=0x13105954_0005),
}

# cfg4: the six serving instances (lenslets, m, precision)
SERVING_INSTANCES = [(20, 32, PREC_FP32), (40, 32, PREC_FP32), (60, 64, PREC_FP32),
                     (84, 64, PREC_BF16), (84, 64, PREC_BF16), (100, 128, PREC_BF16)]
SERVING_RATES_HZ = [500.0, 800.0, 1000.0, 1200.0, 1500.0, 2000.0]


def serving_config(i: int) -> dict:
    lens, m, prec = SERVING_INSTANCES[i]
    return dict(name=f"cfg4.{i}", lenslets=lens, shape="circular", m=m, window=5 if lens <= 40 else 6,
                stride=3 if lens <= 40 else 4, halo=2, taper=True, min_actuators=0 if lens <= 40 else 8,
                precision=prec, r0=0.12, L0=30.0, layers=[dict(weight=1.0, speed=10.0)], frames=10000,
                seeds=(1313 + i, 5957 + i, 40 + i), philox_seed=0x13105954_0400 + i)


def _speed_fn(spec, frames_total: int):
    if isinstance(spec, tuple) and spec[0] == "ramp":
        _, v0, v1, T = spec
        return lambda t: v0 + (v1 - v0) * min(max(t / T, 0.0), 1.0)
    return float(spec)


@dataclass
class Case:
    cfg: dict
    geom: Geometry
    D: CSR
    dmap: DomainMap
    m: int
    a1: np.ndarray
    a2: np.ndarray
    sigma_v: float
    r_inv: np.ndarray
    inflation: float
    philox_seed: int
    X0: np.ndarray          # (n, m): rows [phi_0 ; phi_-1] on the actuators
    truth: FrozenFlow
    noise_seed: int
    precision: int

    @property
    def n_act(self):
        return self.geom.n_act

    @property
    def n_sub(self):
        return self.geom.n_sub

    def truth_phase(self, k: int) -> np.ndarray:
        return self.truth.phase(k * DT)

    def slopes(self, k: int) -> np.ndarray:
        """Measured slopes of frame k: D phi_k + N(0, SIGMA^2)."""
        phi = self.truth_phase(k)
        y = self.D.to_dense() @ phi if self.geom.n_act < 400 else _csr_mv(self.D, phi)
        rng = np.random.default_rng([self.noise_seed, k])
        return y + SIGMA * rng.standard_normal(len(y))


def _csr_mv(D: CSR, v: np.ndarray) -> np.ndarray:
    rows = np.repeat(np.arange(D.shape[0]), np.diff(D.rowptr))
    return np.bincount(rows, weights=D.val * v[D.col], minlength=D.shape[0])


def build_case(cfg, m: int | None = None, precision: int | None = None, dmap: DomainMap | None = None,
               global_map: bool = False, sigma_v: float | None = None, partitions: int = 1) -> Case:
    """partitions = 2: the workload's window partition plus one staggered by
    half a stride, averaged (both run in the same analysis launch)."""
    if isinstance(cfg, int):
        cfg = CONFIGS[cfg]
    cfg = dict(cfg)
    m = int(m or cfg["m"])
    geom = build_geometry(cfg["lenslets"], cfg["shape"])
    D = fried_slope_matrix(geom)
    if dmap is None:
        if global_map:
            dmap = global_domain(geom)
        else:
            parts = [window_domains(geom, cfg["window"], cfg["stride"], cfg["halo"], cfg["taper"],
                                    cfg["min_actuators"], shift=(k * cfg["stride"]) // partitions)
                     for k in range(partitions)]
            dmap = parts[0] if partitions == 1 else combine_maps(parts)
    act_xy = geom.act_rc[:, ::-1].astype(float) * PITCH  # (x = column, y = row)
    screen_seed, noise_seed, ens_seed = cfg["seeds"]
    layers = [dict(L, speed=_speed_fn(L["speed"], cfg["frames"])) for L in cfg["layers"]]
    vmax = max(max(L["speed"][1], L["speed"][2]) if isinstance(L["speed"], tuple) else L["speed"]
               for L in cfg["layers"])
    travel = vmax * cfg["frames"] * DT
    truth = FrozenFlow(act_xy, cfg["r0"], cfg["L0"], layers, travel, screen_seed, pitch=PITCH)
    v0 = layers[0]["speed"](0.0) if callable(layers[0]["speed"]) else layers[0]["speed"]
    # the members need von Karman statistics at the actuator points only, so their
    # screens use two pixels per pitch (the truth keeps four for the slopes)
    phi0, phim1 = independent_screens_at(act_xy, cfg["r0"], cfg["L0"], m, ens_seed, v0 * DT, oversample=2,
                                         pitch=PITCH)
    X0 = np.vstack([phi0, phim1])
    if sigma_v is None:
        ph = truth.phase(0.0)
        sigma_v = float(np.sqrt(np.var(ph) / ar2_stationary_gain(A1, A2)))
    n_act = geom.n_act
    return Case(cfg=cfg, geom=geom, D=D, dmap=dmap, m=m, a1=np.full(n_act, A1), a2=np.full(n_act, A2),
                sigma_v=sigma_v, r_inv=np.full(geom.p, 1.0 / SIGMA ** 2), inflation=1.0,
                philox_seed=int(cfg["philox_seed"]), X0=X0, truth=truth, noise_seed=noise_seed,
                precision=cfg["precision"] if precision is None else precision)
