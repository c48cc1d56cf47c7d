"""Local ETKF analysis and AR forecast, float64, one step at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State (paper Sec. 2.1): x_k holds two successive instants of the phase on the
valid actuators, so n = 2 n_act; here the rows are [phi_k ; phi_{k-1}].
Observations y_k are the x then y slopes of the valid subapertures, p = 2 n_sub,
through the WFS matrix D (Sec. 3), observing the current instant: H = [D 0].

Ensemble (Sec. 2.2): m members, columns of X (n x m); the covariances are the
empirical ones, which the ETKF never forms.

Local ETKF (Sec. 2.3, ref [14]): each estimation domain l (actuators E_l,
both instants) is updated from its observation region O_l (both slopes of
each subaperture) independently of the others.  In ensemble space, with
r = taper * R^-1 on O_l and inflation rho (1 = none):
    C      = Y'_O^T diag(r) Y'_O                 (m x m)
    b      = Y'_O^T diag(r) d_O,   d = y - ybar  (m)
    A      = (m-1)/rho I + C  =  U Lambda U^T    (eigh)
    P~     = A^-1,   wbar = P~ b
    W      = [(m-1) P~]^(1/2)  (symmetric square root, ref [9])
    Z      = xbar_E 1^T + X'_E (W + wbar 1^T)
The whole-pupil analysis (Sec. 3.2) merges the domain estimates row by row
with weights omega (sum over the domains covering a row = 1).

Forecast (Sec. 2.1, AR(1) or AR(2) with a2 = 0 giving AR(1)):
    phi_{k+1} = a1 * phi_k + a2 * phi_{k-1} + sigma_v z,   z ~ N(0, I)
and the new state is [phi_{k+1} ; phi_k].
"""
from __future__ import annotations

import numpy as np

from .philox import forecast_normals


def ensemble_mean_perturbations(X: np.ndarray):
    """xbar = X 1 / m and X' = X - xbar 1^T  (Sec. 2.2)."""
    xbar = X.mean(axis=1)
    return xbar, X - xbar[:, None]


def slope_synthesis(D: np.ndarray, X: np.ndarray, n_act: int):
    """Slopes of each member through H = [D 0]: returns ybar (p) and Y' (p x m)."""
    Y = D @ X[:n_act]
    ybar = Y.mean(axis=1)
    return ybar, Y - ybar[:, None]


def domain_analysis(Xp_E: np.ndarray, xbar_E: np.ndarray, Yp_O: np.ndarray, d_O: np.ndarray,
                    r_O: np.ndarray, rho: float = 1.0) -> dict:
    """One domain's ensemble-space update (Sec. 2.3, refs [9], [14])."""
    m = Xp_E.shape[1]
    C = Yp_O.T @ (r_O[:, None] * Yp_O)
    b = Yp_O.T @ (r_O * d_O)
    A = (m - 1) / rho * np.eye(m) + C
    lam, U = np.linalg.eigh(A)
    wbar = U @ ((U.T @ b) / lam)
    W = (U * np.sqrt((m - 1) / lam)) @ U.T
    T = W + wbar[:, None]
    Z = xbar_E[:, None] + Xp_E @ T
    return dict(C=C, b=b, A=A, lam=lam, U=U, wbar=wbar, W=W, T=T, Z=Z)


def domain_rows(dmap, l: int, n_act: int, n_sub: int):
    """State rows (both instants) and slope rows (x and y) of domain l."""
    E = np.asarray(dmap.est(l), dtype=np.int64)
    O = np.asarray(dmap.obs(l), dtype=np.int64)
    state_rows = np.concatenate([E, n_act + E])
    obs_rows = np.concatenate([O, n_sub + O])
    return E, O, state_rows, obs_rows


def analysis(X: np.ndarray, y: np.ndarray, D: np.ndarray, dmap, r_inv: np.ndarray,
             rho: float = 1.0, keep_domains: bool = False):
    """Whole-pupil local ETKF analysis of the forecast ensemble X (n x m)."""
    n, m = X.shape
    n_act = n // 2
    p = D.shape[0]
    n_sub = p // 2
    xbar, Xp = ensemble_mean_perturbations(X)
    ybar, Yp = slope_synthesis(D, X, n_act)
    d = y - ybar
    Xa = np.zeros_like(X)
    per_domain = []
    for l in range(dmap.n_domains):
        E, O, srows, orows = domain_rows(dmap, l, n_act, n_sub)
        taper = np.asarray(dmap.taper(l), dtype=float)
        r_O = np.concatenate([taper, taper]) * r_inv[orows]
        res = domain_analysis(Xp[srows], xbar[srows], Yp[orows], d[orows], r_O, rho)
        w = np.asarray(dmap.weights(l), dtype=float)
        Xa[srows] += np.concatenate([w, w])[:, None] * res["Z"]
        if keep_domains:
            per_domain.append(res)
    return (Xa, per_domain) if keep_domains else Xa


def forecast(Xa: np.ndarray, a1: np.ndarray, a2: np.ndarray, sigma_v: float, seed: int,
             frame: int) -> np.ndarray:
    """AR(2) forecast of the analysis ensemble (Sec. 2.1)."""
    n, m = Xa.shape
    n_act = n // 2
    phi_k, phi_km1 = Xa[:n_act], Xa[n_act:]
    phi_next = a1[:, None] * phi_k + a2[:, None] * phi_km1
    if sigma_v != 0.0:
        phi_next = phi_next + sigma_v * forecast_normals(seed, frame, n_act, m)
    return np.vstack([phi_next, phi_k])


def frame_step(Xf: np.ndarray, y: np.ndarray, D: np.ndarray, dmap, r_inv, a1, a2, sigma_v,
               seed: int, frame: int, rho: float = 1.0):
    """Analysis of frame k then forecast to k+1; returns (X^a, X^f_{k+1})."""
    Xa = analysis(Xf, y, D, dmap, r_inv, rho)
    return Xa, forecast(Xa, a1, a2, sigma_v, seed, frame)
