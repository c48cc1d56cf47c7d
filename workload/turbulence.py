"""Seeded von Karman phase screens with Taylor frozen flow (paper Sec. 3).

Input synthesis only: the truth phase at the actuator points, the measured
slopes and the initial ensemble.  Screens are periodic FFT screens: complex
Gaussian noise filtered by the von Karman phase PSD
    Phi(f) = 0.023 r0^(-5/3) (f^2 + L0^-2)^(-11/6)   [rad^2 m^2]
(the standard FFT phase-screen recipe), sampled on a square grid of pixel
``delta`` metres and read at arbitrary points by periodic bilinear
interpolation, so that a layer moving at velocity v is read at x + v t.
"""
from __future__ import annotations

import numpy as np


def von_karman_screen(npix: int, delta: float, r0: float, L0: float,
                      rng: np.random.Generator) -> np.ndarray:
    fx = np.fft.fftfreq(npix, d=delta)
    f2 = fx[None, :] ** 2 + fx[:, None] ** 2
    psd = 0.023 * r0 ** (-5.0 / 3.0) * (f2 + 1.0 / L0 ** 2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    df = 1.0 / (npix * delta)
    cn = (rng.standard_normal((npix, npix)) + 1j * rng.standard_normal((npix, npix))) * np.sqrt(psd) * df
    return np.real(np.fft.ifft2(cn)) * npix * npix


def sample_bilinear(screen: np.ndarray, delta: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Periodic bilinear read of ``screen`` at metric points (x, y)."""
    npix = screen.shape[0]
    u = np.asarray(x, float) / delta
    v = np.asarray(y, float) / delta
    u0 = np.floor(u)
    v0 = np.floor(v)
    fu = u - u0
    fv = v - v0
    i0 = v0.astype(np.int64) % npix
    j0 = u0.astype(np.int64) % npix
    i1 = (i0 + 1) % npix
    j1 = (j0 + 1) % npix
    return ((1 - fv) * ((1 - fu) * screen[i0, j0] + fu * screen[i0, j1])
            + fv * ((1 - fu) * screen[i1, j0] + fu * screen[i1, j1]))


class FrozenFlow:
    """Sum of frozen-flow von Karman layers read at the actuator points.

    layers: list of dicts {weight, speed(t)->m/s or float, angle_deg}; the
    layer r0 is r0 * weight^(-3/5) so the Cn^2 weights add up to r0."""

    def __init__(self, act_xy: np.ndarray, r0: float, L0: float, layers, travel_m: float,
                 seed: int, oversample: int = 4, pitch: float = 0.5):
        self.act_xy = np.asarray(act_xy, float)
        self.delta = pitch / oversample
        extent = float(self.act_xy.max()) + pitch
        need = 2.0 * (extent + travel_m)
        npix = 64
        while npix * self.delta < need:
            npix *= 2
        rng = np.random.default_rng(seed)
        self.layers = []
        for L in layers:
            r0_l = r0 * L["weight"] ** (-3.0 / 5.0)
            scr = von_karman_screen(npix, self.delta, r0_l, L0, rng)
            self.layers.append(dict(screen=scr, speed=L["speed"], angle=np.deg2rad(L.get("angle_deg", 0.0))))

    def position(self, layer, t: float) -> float:
        sp = layer["speed"]
        if callable(sp):
            # integrate speed(t) with a fine trapezoid (monotone ramps only need a few points)
            ts = np.linspace(0.0, t, 65) if t > 0 else np.array([0.0, t])
            vs = np.array([sp(tt) for tt in ts])
            return float(np.sum(0.5 * (vs[1:] + vs[:-1]) * np.diff(ts)))
        return float(sp) * t

    def phase(self, t: float) -> np.ndarray:
        return self.phase_at(self.act_xy, t)

    def phase_at(self, xy: np.ndarray, t: float) -> np.ndarray:
        """The same screens read at other metric points (inside the pupil)."""
        xy = np.asarray(xy, float)
        out = np.zeros(len(xy))
        for L in self.layers:
            s = self.position(L, t)
            dx, dy = s * np.cos(L["angle"]), s * np.sin(L["angle"])
            out += sample_bilinear(L["screen"], self.delta, xy[:, 0] + dx, xy[:, 1] + dy)
        return out


def independent_screens_at(act_xy: np.ndarray, r0: float, L0: float, count: int, seed: int,
                           shift_m: float, oversample: int = 4, pitch: float = 0.5):
    """``count`` independent single-layer screens read at the actuators at
    t = 0 and shifted by ``shift_m`` along x (one frame of travel back in
    time).  Returns two (n_act, count) arrays (phi(0), phi(-dt))."""
    act_xy = np.asarray(act_xy, float)
    delta = pitch / oversample
    extent = float(act_xy.max()) + pitch
    npix = 64
    while npix * delta < 2.0 * (extent + abs(shift_m) + pitch):
        npix *= 2
    rng = np.random.default_rng(seed)
    a = np.zeros((len(act_xy), count))
    b = np.zeros((len(act_xy), count))
    for k in range(count):
        scr = von_karman_screen(npix, delta, r0, L0, rng)
        a[:, k] = sample_bilinear(scr, delta, act_xy[:, 0], act_xy[:, 1])
        b[:, k] = sample_bilinear(scr, delta, act_xy[:, 0] - shift_m, act_xy[:, 1])
    return a, b
