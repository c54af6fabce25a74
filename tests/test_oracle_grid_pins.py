"""Pins of the grid-construction oracle (Eq. scene-norm, Eq. voxel-size)
against brute force, pure-Python statistics, numpy's percentile and closed-form
scenes.  CPU only."""
import math
import random
import statistics

import numpy as np
import pytest

from oracle import grid_stats as G


def test_order_statistics_match_brute_force_sorting():
    rng = random.Random(5)
    for n in (1, 2, 3, 7, 64, 101):
        vals = [float(rng.choice([-2.5, 0.0, 1.0, 3.25, rng.uniform(-5, 5)])) for _ in range(n)]
        srt = sorted(vals)
        a = np.asarray(vals)
        for k in range(n):
            assert G.order_stat(a, k) == srt[k]


def test_median_matches_pure_python_statistics():
    rng = random.Random(9)
    for n in (1, 2, 5, 6, 99, 100):
        vals = [rng.uniform(-10, 10) for _ in range(n)]
        assert G.median(np.asarray(vals)) == statistics.median(vals)


def test_percentile_matches_numpy_within_rounding_and_exact_on_integers():
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 10, 1000, 4097):
        v = rng.standard_normal(n) * 3.0
        ref = float(np.percentile(v, 99.0, method="linear"))
        got = G.percentile_linear(v, 0.99)
        assert abs(got - ref) <= 4 * np.spacing(abs(ref) + 1.0)
    # 0..100: the 99th percentile is 99 exactly; 0..1000 at q = 0.5 is 500
    assert G.percentile_linear(np.arange(101, dtype=np.float64), 0.99) == 99.0
    assert G.percentile_linear(np.arange(1001, dtype=np.float64)[::-1].copy(), 0.5) == 500.0
    # interpolation: [0, 10] at q = 0.99 -> 9.9 (0.99 * 10 in binary64)
    assert G.percentile_linear(np.array([10.0, 0.0]), 0.99) == 0.0 + (10.0 - 0.0) * 0.99


def test_next_power_of_two_rule():
    assert G.next_pow2_at_least(0.3, 512) == 2
    assert G.next_pow2_at_least(2.0, 512) == 2
    assert G.next_pow2_at_least(2.0000001, 512) == 4
    assert G.next_pow2_at_least(26.67, 512) == 32
    assert G.next_pow2_at_least(512.0, 512) == 512
    assert G.next_pow2_at_least(682.7, 512) == 512
    assert G.next_pow2_at_least(682.7, 1024) == 1024


def _star_scene(copies=100, floaters=5):
    """Six axis tips at distance 3 around c = (1, -2, 0.5), repeated, plus a
    few far floaters along +x: every statistic has a closed form."""
    c = np.array([1.0, -2.0, 0.5])
    tips = np.array([[3, 0, 0], [-3, 0, 0], [0, 3, 0], [0, -3, 0], [0, 0, 3], [0, 0, -3]], dtype=np.float64)
    pts = np.concatenate([c + tips] * copies + [np.tile(c + np.array([100.0, 0, 0]), (floaters, 1))])
    return c, pts.astype(np.float32)


def test_closed_form_star_scene_without_scales():
    c, pts = _star_scene()
    r = G.grid_from_points(pts, None, g_max=512)
    assert r["center"] == list(c)          # medians of symmetric coordinates
    assert r["r_fg"] == 3.0                # the floaters are in the top 1 %
    assert r["b"] == 4.0                   # ceil(1.05 * 3) = ceil(3.15)
    assert r["h_v"] == 3.0 / 256
    assert r["dim"] == 512                 # 2 b / h_v = 682.7 -> 1024, capped
    assert r["voxel"] == 8.0 / 512
    assert r["origin"] == [c[0] - 4, c[1] - 4, c[2] - 4]
    assert r["m"] == len(pts)
    assert r["n_kept"] == 600              # the floaters are outside the cube


def test_closed_form_star_scene_with_scales_and_cap():
    c, pts = _star_scene()
    s = np.full(len(pts), 0.1, dtype=np.float32)
    r = G.grid_from_points(pts, s, g_max=1024)
    assert r["s_med"] == float(np.float32(0.1))
    assert r["h_v"] == 3.0 * float(np.float32(0.1))
    assert r["dim"] == 32                  # 8 / 0.3 = 26.7
    assert r["voxel"] == 8.0 / 32
    # tiny scales: the scene term wins and the cap applies
    r2 = G.grid_from_points(pts, np.full(len(pts), 1e-6, dtype=np.float32), g_max=1024)
    assert r2["h_v"] == 3.0 / 256 and r2["dim"] == 1024


def test_non_finite_points_do_not_take_part():
    c, pts = _star_scene()
    bad = np.array([[np.nan, 0, 0], [0, np.inf, 0], [1e30, 1e30, -np.inf]], dtype=np.float32)
    r0 = G.grid_from_points(pts, None)
    r1 = G.grid_from_points(np.concatenate([pts, bad]), None)
    for k in ("center", "r_fg", "b", "h_v", "dim", "origin", "voxel", "n_kept"):
        assert r0[k] == r1[k], k
    assert r1["m"] == r0["m"]
    # a NaN scale removes the point from every statistic
    s = np.full(len(pts) + 1, 0.1, dtype=np.float32)
    s[-1] = np.nan
    r2 = G.grid_from_points(np.concatenate([pts, pts[:1]]), s)
    assert r2["m"] == len(pts)


def test_even_count_median_is_mean_of_middles_and_kept_rule_at_the_faces():
    pts = np.array([[0, 0, 0], [2, 2, 2], [4, 4, 4], [6, 6, 6]], dtype=np.float32)
    r = G.grid_from_points(pts, None, g_max=4)
    assert r["center"] == [3.0, 3.0, 3.0]
    # distances sqrt(27), sqrt(3), sqrt(3), sqrt(27); P99 at position 2.97
    d = sorted([math.sqrt(27.0), math.sqrt(3.0), math.sqrt(3.0), math.sqrt(27.0)])
    assert r["r_fg"] == d[2] + (d[3] - d[2]) * (0.99 * 3 - 2)
    assert r["b"] == float(math.ceil(1.05 * math.sqrt(27.0)))   # 6
    # the grid is [3 - 6, 3 + 6)^3; every point is inside
    assert r["n_kept"] == 4
    # a point on the upper face is outside, one on the lower face inside
    lo = np.array([[3.0 - r["b"]] * 3], dtype=np.float32)
    hi = np.array([[3.0 + r["b"]] * 3], dtype=np.float32)
    q_lo = np.floor((lo.astype(np.float64) - np.asarray(r["origin"])) / r["voxel"])
    q_hi = np.floor((hi.astype(np.float64) - np.asarray(r["origin"])) / r["voxel"])
    assert np.all(q_lo == 0) and np.all(q_hi == r["dim"])


def test_degenerate_inputs_raise():
    with pytest.raises(ValueError):
        G.grid_from_points(np.full((4, 3), np.nan, dtype=np.float32))
    with pytest.raises(ValueError):
        G.grid_from_points(np.zeros((10, 3), dtype=np.float32))   # zero extent
