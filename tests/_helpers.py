"""Shared helpers of the test-suite (not collected by pytest)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import oracle
from workload.configs import build_case  # noqa: F401  (re-export)


def sparse_D(case):
    return sp.csr_matrix((case.D.val, case.D.col, case.D.rowptr), shape=case.D.shape)


def rel(a, b):
    """Normwise relative error ||a - b||_F / ||b||_F."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rowmax(a, b, floor=1e-3):
    """Largest per-row relative error: max over rows i of ||a_i - b_i|| /
    max(||b_i||, floor x RMS row norm of b) (rows: last axis for 2-D arrays,
    single values for vectors).  Unlike the Frobenius ratio, one bad domain's
    rows cannot hide among thousands of good ones."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    rms = float(np.sqrt(np.mean(den ** 2))) if den.size else 0.0
    den = np.maximum(den, floor * rms if rms > 0 else 1.0)
    return float(np.max(num / den)) if num.size else 0.0


def split(X):
    """(mean, perturbations) of an ensemble matrix."""
    mu = X.mean(axis=1)
    return mu, X - mu[:, None]


def oracle_spin_up(case, frames: int, X=None):
    """Run the oracle from X0 for `frames` frames; returns the forecast
    ensemble entering frame `frames` (and that frame index)."""
    D = sparse_D(case)
    X = case.X0.copy() if X is None else X
    for k in range(frames):
        Xa = oracle.analysis(X, case.slopes(k), D, case.dmap, case.r_inv, case.inflation)
        X = oracle.forecast(Xa, case.a1, case.a2, case.sigma_v, case.philox_seed, k)
    return X, frames


def result_errors(G_a, O_a, G_f=None, O_f=None):
    """Per-result errors: normwise (analysis mean, analysis perturbations,
    forecast) and the largest per-row ones (mean_row, pert_row)."""
    gm, gp = split(G_a)
    om, op = split(O_a)
    # mean_row: each actuator's error against max(|value|, RMS of the mean): the
    # mean phase crosses zero, where a purely relative error means nothing.
    # ens_row: each state row of the analysis ensemble (mean and perturbations)
    # against max(its norm, the RMS row norm), for the same reason.  pert_row: each row's perturbations against their
    # own norm; with an FP32 ensemble this is bounded by the storage rounding
    # of rows whose mean is 1e4-1e5 times their spread, not by the kernels.
    out = dict(mean=rel(gm, om), pert=rel(gp, op), mean_row=rowmax(gm, om, floor=1.0),
               ens_row=rowmax(G_a, O_a, floor=1.0), pert_row=rowmax(gp, op))
    if G_f is not None:
        out["forecast"] = rel(G_f, O_f)
    return out
