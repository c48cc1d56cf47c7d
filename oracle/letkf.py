"""Local ETKF analysis and AR forecast, float64, one step at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State (paper Sec. 2.1): x_k holds two successive instants of the phase on the
valid actuators, so n = 2 n_act; here the rows are [phi_k ; phi_{k-1}].
Observations y_k are the x then y slopes of the valid subapertures, p = 2 n_sub,
through the WFS matrix D (Sec. 3), observing one of the two instants the state
holds: the current one, H = [D 0] (obs_instant = 0), or the previous one,
H = [0 D] (obs_instant = 1).

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

Differential pistons (Sec. 3.2): slopes do not see a constant phase, and each
domain is estimated on its own, so the domain estimates disagree by a
constant ("differential pistons"), which a post-processing step removes before
the whole-pupil reconstruction.  The paper does not describe its method; the
reading here: each domain's rows of instant t (phi_k or phi_{k-1}) and member
i are shifted by one constant c_l[t, i] chosen by least squares so that the
domains agree on the actuators they share,
    minimise  sum_j  sum_{l < l' covering j} (Z_l[j] + c_l - Z_l'[j] - c_l')^2,
taking the minimum-norm solution and then the constant that leaves the merged
sum of each member's phase unchanged (sum_l w_l c_l = 0, w_l = sum of domain
l's merge weights).

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


def slope_synthesis(D: np.ndarray, X: np.ndarray, n_act: int, obs_instant: int = 0):
    """Slopes of each member through H = [D 0] (obs_instant 0) or H = [0 D]
    (obs_instant 1): returns ybar (p) and Y' (p x m)."""
    Y = D @ X[obs_instant * n_act:(obs_instant + 1) * n_act]
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


def domain_pistons(Zs: list, dmap, n_act: int) -> np.ndarray:
    """Least-squares differential pistons c[l, t, i] of the domain estimates
    Zs[l] (rows: the domain's actuators at phi_k, then at phi_{k-1}), as read
    in the module docstring.  Pairs of domains sharing an actuator, one term
    per shared actuator, are accumulated into the normal equations
    Lap c = r of the objective; numpy's pseudo-inverse gives the minimum-norm
    solution."""
    L = dmap.n_domains
    m = Zs[0].shape[1] if L else 0
    cover = [[] for _ in range(n_act)]
    for l in range(L):
        for pos, j in enumerate(dmap.est(l)):
            cover[int(j)].append((l, pos))
    lap = np.zeros((L, L))
    r = np.zeros((L, 2, m))
    for j in range(n_act):
        for a, pa in cover[j]:
            ea = len(dmap.est(a))
            for b, pb in cover[j]:
                if a == b:
                    continue
                eb = len(dmap.est(b))
                lap[a, a] += 1.0
                lap[a, b] -= 1.0
                for t in (0, 1):
                    r[a, t] += Zs[b][t * eb + pb] - Zs[a][t * ea + pa]
    c = np.einsum("lk,ktm->ltm", np.linalg.pinv(lap), r)
    w = np.array([np.sum(dmap.weights(l)) for l in range(L)])
    c -= np.einsum("l,ltm->tm", w, c)[None] / w.sum()
    return c


def analysis(X: np.ndarray, y: np.ndarray, D: np.ndarray, dmap, r_inv: np.ndarray,
             rho: float = 1.0, keep_domains: bool = False, pistons: bool = False, obs_instant: int = 0):
    """Whole-pupil local ETKF analysis of the forecast ensemble X (n x m);
    pistons: remove the differential pistons before the merge; obs_instant:
    the instant the slopes observe (0: phi_k, 1: phi_{k-1})."""
    n, m = X.shape
    n_act = n // 2
    p = D.shape[0]
    n_sub = p // 2
    xbar, Xp = ensemble_mean_perturbations(X)
    ybar, Yp = slope_synthesis(D, X, n_act, obs_instant)
    d = y - ybar
    Xa = np.zeros_like(X)
    per_domain = []
    for l in range(dmap.n_domains):
        E, O, srows, orows = domain_rows(dmap, l, n_act, n_sub)
        taper = np.asarray(dmap.taper(l), dtype=float)
        r_O = np.concatenate([taper, taper]) * r_inv[orows]
        per_domain.append(domain_analysis(Xp[srows], xbar[srows], Yp[orows], d[orows], r_O, rho))
    c = domain_pistons([res["Z"] for res in per_domain], dmap, n_act) if pistons else None
    for l, res in enumerate(per_domain):
        E, O, srows, orows = domain_rows(dmap, l, n_act, n_sub)
        w = np.asarray(dmap.weights(l), dtype=float)
        Z = res["Z"]
        if pistons:
            e = len(E)
            Z = Z + np.concatenate([np.repeat(c[l, 0][None], e, 0), np.repeat(c[l, 1][None], e, 0)])
        Xa[srows] += np.concatenate([w, w])[:, None] * Z
    if pistons and keep_domains:
        for l, res in enumerate(per_domain):
            res["piston"] = c[l]
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
               seed: int, frame: int, rho: float = 1.0, obs_instant: int = 0):
    """Analysis of frame k then forecast to k+1; returns (X^a, X^f_{k+1})."""
    Xa = analysis(Xf, y, D, dmap, r_inv, rho, obs_instant=obs_instant)
    return Xa, forecast(Xa, a1, a2, sigma_v, seed, frame)
