"""Pins of the FP64 oracle to closed forms, to the Kalman-filter identity,
to library routines and to brute force (CPU only)."""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import analysis, domain_analysis, forecast, forecast_normals, philox4x32_10
from oracle.letkf import ensemble_mean_perturbations, slope_synthesis
from workload.geometry import (build_geometry, fried_slope_matrix, global_domain, window_domains,
                               DomainMap)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox / noise
def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        out = philox4x32_10(np.array(w[0:4]), np.array(w[4:6]))
        assert [int(v) for v in out] == w[6:10]


def test_box_muller_known_answer():
    """The word -> uniform -> normal map, taken by hand from the published
    Philox4x32-10 answers: u1 = ((x0 2^21 + x1 div 2^11) + 1/2) 2^-53 (one
    rounding to double, exact integer arithmetic here), u2 likewise from
    (x2, x3), z = sqrt(-2 ln u1) cos(2 pi u2) evaluated in 40-digit decimal
    arithmetic.  The uniforms must match bit for bit; the normal within the
    rounding of the double-precision formula, whose angle 2 pi u2 carries an
    absolute error of a few eps (so a bound of 8 eps (r (1 + 2 pi u2) + |z|),
    r = sqrt(-2 ln u1), and not a relative one near a zero of the cosine).  A
    swapped uniform, a sine for the cosine or a dropped factor moves z by O(1)."""
    from decimal import Decimal, getcontext
    from fractions import Fraction
    from oracle.philox import box_muller
    getcontext().prec = 40
    pi40 = Decimal("3.141592653589793238462643383279502884197")

    def cos_dec(x):
        x = x % (2 * pi40)
        term, total, k = Decimal(1), Decimal(1), 0
        while abs(term) > Decimal(10) ** -38:
            k += 2
            term *= -x * x / (k * (k - 1))
            total += term
        return total

    rows = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        x0, x1, x2, x3 = [int(t, 16) for t in line.split()][6:10]
        u1 = float(Fraction(x0 * 2 ** 21 + (x1 >> 11)) + Fraction(1, 2)) * 2.0 ** -53
        u2 = float(Fraction(x2 * 2 ** 21 + (x3 >> 11)) + Fraction(1, 2)) * 2.0 ** -53
        z_exact = (-2 * Decimal(u1).ln()).sqrt() * cos_dec(2 * pi40 * Decimal(u2))
        z = float(box_muller(np.array([[x0, x1, x2, x3]], dtype=np.uint32))[0])
        # the oracle's uniforms, recomputed from its own arithmetic, bit for bit
        v1 = (np.uint64(x0) << np.uint64(21)) | (np.uint64(x1) >> np.uint64(11))
        assert (float(v1) + 0.5) * 2.0 ** -53 == u1
        r = float((-2 * Decimal(u1).ln()).sqrt())
        bound = 8 * 2.0 ** -52 * (r * (1 + 2 * np.pi * u2) + abs(float(z_exact)))
        assert abs(z - float(z_exact)) <= bound, (z, z_exact, bound)
        rows += 1
    assert rows >= 3


def test_forecast_normals_are_standard_normal():
    z = forecast_normals(seed=12345, frame=7, n_act=500, m=128).ravel()
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.02
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # distinct frames / seeds / members give independent streams
    z2 = forecast_normals(seed=12345, frame=8, n_act=500, m=128).ravel()
    z3 = forecast_normals(seed=12346, frame=7, n_act=500, m=128).ravel()
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.02 and abs(np.corrcoef(z, z3)[0, 1]) < 0.02
    # counter layout: member j of actuator a does not alias actuator j member a
    zz = forecast_normals(seed=1, frame=0, n_act=8, m=8)
    assert not np.allclose(zz, zz.T)


def test_forecast_normals_large_frame_uses_high_word():
    a = forecast_normals(seed=3, frame=5, n_act=4, m=4)
    b = forecast_normals(seed=3, frame=5 + (1 << 32), n_act=4, m=4)
    assert not np.allclose(a, b)


# ---------------------------------------------------------------- helpers
def _rand_domain(rng, m, nE, pO, scale=1.0):
    Xp = rng.standard_normal((nE, m)) * scale
    Xp -= Xp.mean(axis=1, keepdims=True)
    Yp = rng.standard_normal((pO, m)) * scale
    Yp -= Yp.mean(axis=1, keepdims=True)
    return Xp, rng.standard_normal(nE), Yp, rng.standard_normal(pO), rng.uniform(0.5, 2.0, pO)


# ---------------------------------------------------------------- closed forms
def test_m2_closed_form():
    """m = 2, X' = [u, -u], Y' = [v, -v]: mean gain 2uc/(1+2s), spread (1+2s)^-1/2."""
    rng = np.random.default_rng(0)
    u = rng.standard_normal(5)
    v = rng.standard_normal(7)
    d = rng.standard_normal(7)
    r = rng.uniform(0.5, 3, 7)
    xbar = rng.standard_normal(5)
    s = v @ (r * v)
    c = v @ (r * d)
    res = domain_analysis(np.stack([u, -u], 1), xbar, np.stack([v, -v], 1), d, r)
    mean_a = res["Z"].mean(axis=1)
    np.testing.assert_allclose(mean_a, xbar + 2 * u * c / (1 + 2 * s), rtol=1e-13, atol=1e-13)
    pert = res["Z"] - mean_a[:, None]
    np.testing.assert_allclose(pert, np.stack([u, -u], 1) / np.sqrt(1 + 2 * s), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(np.sort(res["lam"]), [1.0, 1 + 2 * s], rtol=1e-13)


def test_scalar_kalman_filter():
    """n = p = 1, H = 1: mean x + P/(P+R) d, variance P R / (P + R)."""
    rng = np.random.default_rng(1)
    for m in (3, 10, 40):
        x = rng.standard_normal(m) * 2.0 + 1.0
        xbar, xp = x.mean(), x - x.mean()
        R = 0.7
        y = 0.3
        P = xp @ xp / (m - 1)
        res = domain_analysis(xp[None, :], np.array([xbar]), xp[None, :], np.array([y - xbar]),
                              np.array([1.0 / R]))
        za = res["Z"][0]
        np.testing.assert_allclose(za.mean(), xbar + P / (P + R) * (y - xbar), rtol=1e-13)
        np.testing.assert_allclose(np.var(za, ddof=1), P * R / (P + R), rtol=1e-12)


def test_no_observations_is_identity():
    rng = np.random.default_rng(2)
    Xp, xbar, Yp, d, r = _rand_domain(rng, 12, 6, 9)
    res = domain_analysis(Xp, xbar, Yp, d, np.zeros_like(r))
    np.testing.assert_allclose(res["W"], np.eye(12), atol=1e-14)
    np.testing.assert_allclose(res["wbar"], 0, atol=1e-15)
    np.testing.assert_allclose(res["Z"], xbar[:, None] + Xp, atol=1e-14)


# ---------------------------------------------------------------- library routines
@pytest.mark.parametrize("m", [2, 3, 4, 7])
def test_tiny_against_sqrtm_and_solve(m):
    rng = np.random.default_rng(10 + m)
    Xp, xbar, Yp, d, r = _rand_domain(rng, m, 3, 5)
    res = domain_analysis(Xp, xbar, Yp, d, r)
    A = (m - 1) * np.eye(m) + Yp.T @ np.diag(r) @ Yp           # brute force
    np.testing.assert_allclose(res["A"], A, rtol=1e-14, atol=1e-13)
    W = scipy.linalg.sqrtm((m - 1) * np.linalg.inv(A)).real
    np.testing.assert_allclose(res["W"], W, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(res["wbar"], scipy.linalg.solve(A, Yp.T @ (r * d)), rtol=1e-11, atol=1e-13)
    # brute-force update, element by element
    T = W + res["wbar"][:, None]
    Z = np.array([[xbar[i] + sum(Xp[i, k] * T[k, j] for k in range(m)) for j in range(m)]
                  for i in range(Xp.shape[0])])
    np.testing.assert_allclose(res["Z"], Z, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("rho", [1.0, 1.05])
def test_transform_invariants(rho):
    rng = np.random.default_rng(3)
    m = 24
    Xp, xbar, Yp, d, r = _rand_domain(rng, m, 10, 30, scale=3.0)
    res = domain_analysis(Xp, xbar, Yp, d, r, rho=rho)
    W, wbar, lam = res["W"], res["wbar"], res["lam"]
    one = np.ones(m)
    np.testing.assert_allclose(W, W.T, atol=1e-14)
    np.testing.assert_allclose(W @ one, one * np.sqrt(rho), rtol=1e-12)     # 1 is an eigvec, lambda = (m-1)/rho
    assert abs(one @ wbar) < 1e-12 * np.abs(wbar).sum()
    Pt = np.linalg.inv(res["A"])
    np.testing.assert_allclose(W @ W, (m - 1) * Pt, rtol=1e-10, atol=1e-14)
    assert lam.min() >= (m - 1) / rho * (1 - 1e-12)
    pert = res["Z"] - res["Z"].mean(axis=1, keepdims=True)
    np.testing.assert_allclose(pert.sum(axis=1), 0, atol=1e-10)
    np.testing.assert_allclose(res["Z"].mean(axis=1), xbar + Xp @ wbar, rtol=1e-12, atol=1e-12)


def test_member_permutation_equivariance():
    rng = np.random.default_rng(4)
    geom = build_geometry(6, "square")
    D = fried_slope_matrix(geom).to_dense()
    dm = window_domains(geom, 3, 2, 1)
    m = 9
    X = rng.standard_normal((geom.n, m))
    y = rng.standard_normal(geom.p)
    r_inv = np.full(geom.p, 4.0)
    perm = rng.permutation(m)
    Xa = analysis(X, y, D, dm, r_inv)
    Xa_p = analysis(X[:, perm], y, D, dm, r_inv)
    np.testing.assert_allclose(Xa_p, Xa[:, perm], rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------- Kalman filter identity
def _kf(xbar, P, H, R, y):
    S = H @ P @ H.T + R
    K = np.linalg.solve(S, H @ P).T      # P H^T S^-1  (S symmetric)
    return xbar + K @ (y - H @ xbar), (np.eye(len(xbar)) - K @ H) @ P


def _tiny_case(rng, lenslets=4, m=8):
    geom = build_geometry(lenslets, "square")
    D = fried_slope_matrix(geom).to_dense()
    H = np.hstack([D, np.zeros_like(D)])
    X = rng.standard_normal((geom.n, m)) * 2.0
    y = rng.standard_normal(geom.p)
    R = np.diag(rng.uniform(0.2, 1.0, geom.p))
    return geom, D, H, X, y, R


@pytest.mark.parametrize("obs_instant", [0, 1])
@pytest.mark.parametrize("m", [2, 5, 16])
def test_global_etkf_equals_kf_with_sample_covariance(m, obs_instant):
    """Woodbury: one global domain gives the KF analysis with P = X'X'^T/(m-1),
    with the slopes observing phi_k (H = [D 0]) or phi_{k-1} (H = [0 D]), the
    observation operator written out densely."""
    rng = np.random.default_rng(5 + m)
    geom, D, H, X, y, R = _tiny_case(rng, 4, m)
    if obs_instant:
        H = np.hstack([np.zeros_like(D), D])
    xbar, Xp = ensemble_mean_perturbations(X)
    P = Xp @ Xp.T / (m - 1)
    mean_kf, Pa_kf = _kf(xbar, P, H, R, y)
    Xa = analysis(X, y, D, global_domain(geom), 1.0 / np.diag(R), obs_instant=obs_instant)
    xa, Xap = ensemble_mean_perturbations(Xa)
    np.testing.assert_allclose(xa, mean_kf, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(Xap @ Xap.T / (m - 1), Pa_kf, rtol=1e-9, atol=1e-10)


def test_observed_instant_swaps_with_the_state_rows():
    """Observing phi_{k-1} (H = [0 D]) is observing phi_k of the ensemble
    whose two instants are swapped: the local analysis, domain by domain and
    merged, commutes with the swap."""
    rng = np.random.default_rng(17)
    geom = build_geometry(10, "circular")
    D = fried_slope_matrix(geom).to_dense()
    dm = window_domains(geom, 4, 3, 1, True, 0)
    n_act, m = geom.n_act, 9
    X = rng.standard_normal((geom.n, m))
    y = rng.standard_normal(geom.p)
    r = rng.uniform(0.5, 2.0, geom.p)
    swap = lambda Z: np.vstack([Z[n_act:], Z[:n_act]])
    a1 = analysis(X, y, D, dm, r, obs_instant=1)
    a0 = analysis(swap(X), y, D, dm, r, obs_instant=0)
    np.testing.assert_allclose(a1, swap(a0), rtol=1e-12, atol=1e-12)
    # and it is a different analysis from observing phi_k
    assert np.abs(a1 - analysis(X, y, D, dm, r)).max() > 1e-3


def test_etkf_exact_kf_when_ensemble_spans_covariance():
    """An ensemble whose sample covariance is exactly P gives the exact KF."""
    rng = np.random.default_rng(6)
    geom, D, H, _, y, R = _tiny_case(rng, 3, 8)
    n = geom.n
    m = n + 5
    L = np.linalg.cholesky(np.cov(rng.standard_normal((n, 4 * n))) + 0.1 * np.eye(n))
    P = L @ L.T
    # E: n orthonormal rows orthogonal to the ones vector
    Q, _ = np.linalg.qr(np.hstack([np.ones((m, 1)), rng.standard_normal((m, n))]))
    E = Q[:, 1:n + 1].T
    xbar = rng.standard_normal(n)
    X = xbar[:, None] + np.sqrt(m - 1) * L @ E
    mean_kf, Pa_kf = _kf(xbar, P, H, R, y)
    Xa = analysis(X, y, D, global_domain(geom), 1.0 / np.diag(R))
    xa, Xap = ensemble_mean_perturbations(Xa)
    np.testing.assert_allclose(xa, mean_kf, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(Xap @ Xap.T / (m - 1), Pa_kf, rtol=1e-9, atol=1e-10)


def test_etkf_converges_to_kf_as_m_grows():
    """Linear-Gaussian case: the ETKF mean error vs the exact KF decays like
    m^-1/2 (Sec. 3.1 convergence claim), measured over seeds."""
    rng0 = np.random.default_rng(7)
    geom, D, H, _, y, R = _tiny_case(rng0, 3, 8)
    n = geom.n
    L = np.linalg.cholesky(np.cov(rng0.standard_normal((n, 4 * n))) + 0.1 * np.eye(n))
    P = L @ L.T
    xtrue = rng0.standard_normal(n)
    mean_kf, _ = _kf(xtrue, P, H, R, y)
    errs = []
    ms = [8, 32, 128, 512]
    for m in ms:
        e = []
        for s in range(12):
            rng = np.random.default_rng(1000 * m + s)
            X = xtrue[:, None] + L @ rng.standard_normal((n, m))
            X += (xtrue - X.mean(axis=1))[:, None]           # exact forecast mean
            Xa = analysis(X, y, D, global_domain(geom), 1.0 / np.diag(R))
            e.append(np.linalg.norm(Xa.mean(axis=1) - mean_kf))
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(ms), np.log(errs), 1)[0]
    assert -0.8 < slope < -0.3, (errs, slope)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


# ---------------------------------------------------------------- localization
def test_infinite_halo_domains_equal_global():
    """Every domain seeing every slope without taper uses the global transform,
    so any partition reproduces the global ETKF."""
    rng = np.random.default_rng(8)
    geom = build_geometry(6, "square")
    D = fried_slope_matrix(geom).to_dense()
    m = 10
    X = rng.standard_normal((geom.n, m))
    y = rng.standard_normal(geom.p)
    r_inv = rng.uniform(1, 5, geom.p)
    glob = analysis(X, y, D, global_domain(geom), r_inv)
    for dm in (window_domains(geom, 3, 3, 50), window_domains(geom, 4, 2, 50)):
        np.testing.assert_allclose(analysis(X, y, D, dm, r_inv), glob, rtol=1e-10, atol=1e-10)


def test_merge_weights_average_overlapping_domains():
    """Two identical copies of the global domain with weights 1/2 each give
    the global result (merge is a weighted sum per row)."""
    rng = np.random.default_rng(9)
    geom = build_geometry(5, "square")
    D = fried_slope_matrix(geom).to_dense()
    g = global_domain(geom)
    two = DomainMap(np.array([0, geom.n_act, 2 * geom.n_act], np.int32),
                    np.concatenate([g.est_act, g.est_act]), np.full(2 * geom.n_act, 0.5),
                    np.array([0, geom.n_sub, 2 * geom.n_sub], np.int32),
                    np.concatenate([g.obs_sub, g.obs_sub]), np.ones(2 * geom.n_sub))
    X = rng.standard_normal((geom.n, 6))
    y = rng.standard_normal(geom.p)
    r = np.full(geom.p, 2.0)
    np.testing.assert_allclose(analysis(X, y, D, two, r), analysis(X, y, D, g, r), rtol=1e-12, atol=1e-12)


def test_taper_zero_removes_observation():
    """A zero taper weight is the same as not observing that subaperture."""
    rng = np.random.default_rng(10)
    geom = build_geometry(5, "square")
    D = fried_slope_matrix(geom).to_dense()
    g = global_domain(geom)
    X = rng.standard_normal((geom.n, 7))
    y = rng.standard_normal(geom.p)
    r = np.full(geom.p, 3.0)
    keep = np.arange(geom.n_sub) % 3 != 0
    tap = DomainMap(g.est_ptr, g.est_act, g.est_w, g.obs_ptr, g.obs_sub, keep.astype(float))
    sub = DomainMap(g.est_ptr, g.est_act, g.est_w, np.array([0, keep.sum()], np.int32),
                    g.obs_sub[keep], np.ones(keep.sum()))
    np.testing.assert_allclose(analysis(X, y, D, tap, r), analysis(X, y, D, sub, r), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- slopes / forecast
def test_slope_synthesis_tilt_and_piston():
    geom = build_geometry(8, "circular")
    D = fried_slope_matrix(geom).to_dense()
    c = geom.act_rc[:, 1].astype(float)
    m = 4
    amp = np.array([1.0, -2.0, 0.5, 0.5])
    X = np.vstack([np.outer(c, amp) + 3.0, np.zeros((geom.n_act, m))])   # tilts plus a common piston
    ybar, Yp = slope_synthesis(D, X, geom.n_act)
    np.testing.assert_allclose(ybar[:geom.n_sub], amp.mean())
    np.testing.assert_allclose(Yp[:geom.n_sub], np.tile(amp - amp.mean(), (geom.n_sub, 1)), atol=1e-14)
    np.testing.assert_allclose(Yp[geom.n_sub:], 0, atol=1e-14)


def test_forecast_deterministic_ar2_closed_form():
    """a1 = 1.6, a2 = -0.64 has a double pole at 0.8: phi_k = (c1 + c2 k) 0.8^k."""
    n_act, m = 3, 2
    phi0 = np.array([1.0, -2.0, 0.5])
    phim1 = np.array([0.5, 1.0, 0.0])
    X = np.vstack([np.tile(phi0[:, None], m), np.tile(phim1[:, None], m)])
    a1, a2 = np.full(n_act, 1.6), np.full(n_act, -0.64)
    c1 = phi0
    c2 = c1 - 0.8 * phim1          # from phi_-1 = (c1 - c2) / 0.8
    for k in range(1, 12):
        X = forecast(X, a1, a2, 0.0, seed=0, frame=k)
        np.testing.assert_allclose(X[:n_act, 0], (c1 + c2 * k) * 0.8 ** k, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(X[n_act:, 0], (c1 + c2 * (k - 1)) * 0.8 ** (k - 1), rtol=1e-12, atol=1e-14)


def test_forecast_noise_stationary_variance():
    """AR(2) driven by sigma_v z reaches sigma_v^2 (1-a2)/((1+a2)((1-a2)^2-a1^2))."""
    n_act, m = 200, 64
    a1, a2 = np.full(n_act, 1.6), np.full(n_act, -0.64)
    X = np.zeros((2 * n_act, m))
    acc = []
    for k in range(600):
        X = forecast(X, a1, a2, 1.0, seed=99, frame=k)
        if k >= 200:
            acc.append(np.var(X[:n_act]))
    target = (1 - (-0.64)) / ((1 - 0.64) * ((1 + 0.64) ** 2 - 1.6 ** 2))
    assert abs(np.mean(acc) / target - 1) < 0.06


def test_two_partitions_average_the_two_analyses():
    """Sec. 5 runs two local ETKFs on different domain partitions; read as
    an equal-weight average, one map holding both partitions' domains with
    halved merge weights must give exactly the mean of the two analyses
    (linearity of the weighted merge), and the two partitions must differ."""
    from workload.geometry import combine_maps
    rng = np.random.default_rng(21)
    geom = build_geometry(12, "square")
    D = fried_slope_matrix(geom).to_dense()
    a = window_domains(geom, 4, 4, 1)
    b = window_domains(geom, 4, 4, 1, shift=2)
    assert a.n_domains != b.n_domains or not np.array_equal(a.est_act, b.est_act)
    both = combine_maps([a, b])
    X = rng.standard_normal((geom.n, 8))
    y = rng.standard_normal(geom.p)
    r = np.full(geom.p, 4.0)
    avg = 0.5 * (analysis(X, y, D, a, r) + analysis(X, y, D, b, r))
    np.testing.assert_allclose(analysis(X, y, D, both, r), avg, rtol=1e-12, atol=1e-12)


def _overlapping_square_map(N=10, window=4, stride=3):
    geom = build_geometry(N, "square")
    return geom, window_domains(geom, window, stride, 1)


def test_pistons_reattach_domains_that_differ_by_constants():
    """Domain estimates equal to one field plus an arbitrary constant per
    (domain, instant, member) are re-attached exactly: after the shifts
    every domain carries the same constant, and the weighted sum of the
    shifts is zero (gauge)."""
    from oracle.letkf import domain_pistons
    rng = np.random.default_rng(31)
    geom, dm = _overlapping_square_map()
    m = 5
    f = rng.standard_normal((2, geom.n_act, m))
    k = rng.standard_normal((dm.n_domains, 2, m)) * 3.0
    Zs = []
    for l in range(dm.n_domains):
        E = dm.est(l)
        Zs.append(np.vstack([f[0, E] + k[l, 0], f[1, E] + k[l, 1]]))
    c = domain_pistons(Zs, dm, geom.n_act)
    shifted = k + c                                   # constant left on each domain
    np.testing.assert_allclose(shifted - shifted[:1], 0.0, atol=1e-10)
    w = np.array([dm.weights(l).sum() for l in range(dm.n_domains)])
    np.testing.assert_allclose(np.einsum("l,ltm->tm", w, c), 0.0, atol=1e-10)


def test_pistons_vanish_for_consistent_or_disjoint_domains():
    from oracle.letkf import domain_pistons
    rng = np.random.default_rng(32)
    geom, dm = _overlapping_square_map()
    f = rng.standard_normal((2, geom.n_act, 3))
    Zs = [np.vstack([f[0, dm.est(l)], f[1, dm.est(l)]]) for l in range(dm.n_domains)]
    np.testing.assert_allclose(domain_pistons(Zs, dm, geom.n_act), 0.0, atol=1e-12)
    sq = build_geometry(8, "square")
    disjoint = window_domains(sq, 3, 3, 1)
    Zs = [rng.standard_normal((2 * len(disjoint.est(l)), 3)) for l in range(disjoint.n_domains)]
    np.testing.assert_allclose(domain_pistons(Zs, disjoint, sq.n_act), 0.0, atol=1e-12)


def test_piston_removal_changes_only_the_merged_pistons():
    """On a real analysis the removal moves the merged estimate but keeps each
    member's phase sum (gauge) and leaves a non-overlapping map unchanged."""
    rng = np.random.default_rng(33)
    geom, dm = _overlapping_square_map()
    D = fried_slope_matrix(geom).to_dense()
    X = rng.standard_normal((geom.n, 6))
    y = rng.standard_normal(geom.p)
    r = np.full(geom.p, 4.0)
    a0 = analysis(X, y, D, dm, r)
    a1 = analysis(X, y, D, dm, r, pistons=True)
    assert np.abs(a1 - a0).max() > 1e-6
    np.testing.assert_allclose(a1[:geom.n_act].sum(0), a0[:geom.n_act].sum(0), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(a1[geom.n_act:].sum(0), a0[geom.n_act:].sum(0), rtol=1e-10, atol=1e-10)
    sq = build_geometry(8, "square")
    disjoint = window_domains(sq, 3, 3, 1)
    Dq = fried_slope_matrix(sq).to_dense()
    Xq = rng.standard_normal((sq.n, 4)); yq = rng.standard_normal(sq.p); rq = np.full(sq.p, 4.0)
    np.testing.assert_allclose(analysis(Xq, yq, Dq, disjoint, rq, pistons=True), analysis(Xq, yq, Dq, disjoint, rq),
                               rtol=1e-13, atol=1e-13)
