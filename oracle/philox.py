"""Philox4x32-10 and Box-Muller normals (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x32 is the counter-based generator of Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 128-bit counter is
encrypted under a 64-bit key by R = 10 rounds.  One round maps
(c0, c1, c2, c3) with round key (k0, k1) to
    (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57 (hi/lo = upper/lower 32 bits of the
64-bit product), and the key is bumped by the Weyl constants
(0x9E3779B9, 0xBB67AE85) between rounds.

Forecast model noise (the "stochastic" AR model of Sec. 2.1; the paper does
not give its covariance, so it is sigma_v^2 I on the new time instant):
element (actuator a, member j) of frame f uses
    counter = (j, a, f mod 2^32, f div 2^32),  key = (seed mod 2^32, seed div 2^32)
and the four output words (x0, x1, x2, x3) give two 53-bit uniforms
    u1 = ((x0 * 2^21 + x1 div 2^11) + 1/2) 2^-53,  u2 likewise from (x2, x3)
and one standard normal z = sqrt(-2 ln u1) cos(2 pi u2)  (Box & Muller 1958).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key, rounds: int = 10) -> np.ndarray:
    """counter: (..., 4) uint32-valued array; key: (..., 2).  Returns (..., 4) uint32."""
    c = np.asarray(counter, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(k[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], c0.shape).copy()
    for r in range(rounds):
        p0 = _M0 * c0            # exact: both factors < 2^32, product < 2^64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if r + 1 < rounds:
            k0 = (k0 + np.uint64(_W0)) & _MASK
            k1 = (k1 + np.uint64(_W1)) & _MASK
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def box_muller(words: np.ndarray) -> np.ndarray:
    """Four uint32 words per element -> one standard normal (float64)."""
    w = words.astype(np.uint64)
    v1 = (w[..., 0] << np.uint64(21)) | (w[..., 1] >> np.uint64(11))
    v2 = (w[..., 2] << np.uint64(21)) | (w[..., 3] >> np.uint64(11))
    u1 = (v1.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (v2.astype(np.float64) + 0.5) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def forecast_normals(seed: int, frame: int, n_act: int, m: int) -> np.ndarray:
    """(n_act, m) standard normals of forecast number ``frame``."""
    a = np.arange(n_act, dtype=np.uint64)[:, None]
    j = np.arange(m, dtype=np.uint64)[None, :]
    ctr = np.empty((n_act, m, 4), dtype=np.uint64)
    ctr[..., 0] = j
    ctr[..., 1] = a
    ctr[..., 2] = np.uint64(frame & 0xFFFFFFFF)
    ctr[..., 3] = np.uint64((frame >> 32) & 0xFFFFFFFF)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    return box_muller(philox4x32_10(ctr, key))
