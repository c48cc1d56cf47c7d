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
    """Per-result normwise errors: analysis mean, analysis perturbations, forecast."""
    gm, gp = split(G_a)
    om, op = split(O_a)
    out = dict(mean=rel(gm, om), pert=rel(gp, op))
    if G_f is not None:
        out["forecast"] = rel(G_f, O_f)
    return out
