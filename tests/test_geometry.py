"""Input geometry pinned to the numbers the paper prints (Sec. 3, Sec. 3.2)
and to the properties of the Fried WFS model."""
import os

import numpy as np
import pytest

from workload.geometry import (block_partition, build_geometry, fried_slope_matrix, gaspari_cohn,
                               global_domain, window_domains)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_geometry.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()[:2]
        out[k] = int(v)
    return out


def test_valid_actuator_counts_match_paper():
    g = _golden()
    assert build_geometry(16).n_act == g["act_8m_16x16"]
    g32 = build_geometry(32)
    assert g32.n_act == g["act_16m_32x32"]
    assert g32.n == g["n_16m"] and g32.p == g["p_16m"]


def test_16m_domain_decomposition_matches_paper():
    """7-actuator blocks offset by one with a 3-subaperture halo give the
    Sec. 3.2 numbers: 25 domains, n_max = 98, p_max = 288."""
    g = _golden()
    geom = build_geometry(32)
    st = block_partition(geom, block=7, offset=1, halo=3).stats()
    assert st["n_domains"] == g["domains_16m"]
    assert st["n_max"] == g["nmax_16m"]
    assert st["p_max"] == g["pmax_16m"]
    assert st["sum_n"] == g["n_16m"]          # a partition: every state row once


@pytest.mark.slow
def test_40m_numbers_match_paper_at_threshold_0p6():
    g = _golden()
    geom = build_geometry(80, threshold=0.6, samples=50)
    assert geom.n == g["n_40m"] and geom.p == g["p_40m"]
    st = block_partition(geom, block=9, offset=0, halo=2, min_actuators=5).stats()
    assert st["n_domains"] == g["domains_40m"]
    assert st["n_max"] == g["nmax_40m"]


def test_fried_D_structure():
    geom = build_geometry(12)
    D = fried_slope_matrix(geom).to_dense()
    assert D.shape == (geom.p, geom.n_act)
    assert np.all((D != 0).sum(axis=1) == 4)
    # piston is unseen
    np.testing.assert_allclose(D @ np.ones(geom.n_act), 0, atol=1e-15)
    r, c = geom.act_rc[:, 0].astype(float), geom.act_rc[:, 1].astype(float)
    # a unit tilt along x (column) gives s_x = 1, s_y = 0 everywhere
    s = D @ c
    np.testing.assert_allclose(s[:geom.n_sub], 1.0)
    np.testing.assert_allclose(s[geom.n_sub:], 0.0, atol=1e-15)
    s = D @ r
    np.testing.assert_allclose(s[:geom.n_sub], 0.0, atol=1e-15)
    np.testing.assert_allclose(s[geom.n_sub:], 1.0)
    # the Fried waffle (-1)^(row+col) is in the null space
    np.testing.assert_allclose(D @ (-1.0) ** (r + c), 0, atol=1e-15)


def test_window_map_weights_and_coverage():
    geom = build_geometry(40)
    dm = window_domains(geom, 5, 3, 2, taper=True)
    acc = np.zeros(geom.n_act)
    for l in range(dm.n_domains):
        np.add.at(acc, dm.est(l), dm.weights(l))
    np.testing.assert_allclose(acc, 1.0)
    assert np.all((dm.obs_taper >= 0) & (dm.obs_taper <= 1))
    assert np.all(np.diff(dm.obs_ptr) > 0)


def test_config_maps_match_expected_sizes():
    """Printed (derived) sizes of the three single-instance workloads."""
    sq = build_geometry(15, shape="square")
    assert (sq.n_sub, sq.n_act) == (225, 256)
    st = window_domains(sq, 4, 4, 1).stats()
    assert (st["n_domains"], st["p_max"], st["sum_p"]) == (16, 50, 648)
    g84 = build_geometry(84)
    assert (g84.n_sub, g84.n_act) == (5544, 5713)
    st = window_domains(g84, 6, 4, 2, taper=True, min_actuators=8).stats()
    assert (st["n_domains"], st["e_min"], st["e_max"], st["p_max"]) == (375, 8, 36, 162)


def test_gaspari_cohn_shape():
    z = np.linspace(0, 2.5, 251)
    g = gaspari_cohn(z)
    assert g[0] == 1.0 and np.all(g[z >= 2.0] == 0.0)
    assert np.all(np.diff(g) <= 1e-15)
    # continuity at z = 1 and z = 2 (both branches meet)
    np.testing.assert_allclose(gaspari_cohn(np.array([1 - 1e-9]))[0], gaspari_cohn(np.array([1 + 1e-9]))[0], atol=1e-7)
    assert abs(gaspari_cohn(np.array([2 - 1e-9]))[0]) < 1e-7


def test_global_domain_is_everything():
    geom = build_geometry(6)
    dm = global_domain(geom)
    assert dm.n_domains == 1
    assert len(dm.est(0)) == geom.n_act and len(dm.obs(0)) == geom.n_sub


def test_staggered_partition_covers_and_combines():
    """A partition shifted by half a stride covers every actuator, its window
    corners differ from the unshifted ones, and the combined map's weights
    still sum to one per actuator."""
    from workload.geometry import combine_maps
    g = build_geometry(40)
    a = window_domains(g, 5, 3, 2, taper=True)
    b = window_domains(g, 5, 3, 2, taper=True, shift=1)
    first = {tuple(a.est(l)[:1]) for l in range(a.n_domains)}
    assert any(tuple(b.est(l)[:1]) not in first for l in range(b.n_domains))
    both = combine_maps([a, b])
    assert both.n_domains == a.n_domains + b.n_domains
    acc = np.zeros(g.n_act)
    np.add.at(acc, both.est_act, both.est_w)
    np.testing.assert_allclose(acc, 1.0, rtol=0, atol=1e-14)
