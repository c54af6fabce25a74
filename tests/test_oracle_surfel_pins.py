"""Pins of the needle cull oracle (Eq. aspect, Eq. needle, Eq. pass-needle)
against closed forms, numpy's percentile and counting.  CPU only."""
import numpy as np
import pytest

from oracle import surfel_map as S


def test_aspect_closed_forms():
    s = np.array([[1.0, 1.0], [2.0, 0.5], [0.5, 2.0], [3.0, 0.0]], np.float32)
    a = S.aspect(s)
    assert a[0] == 1.0 / (1.0 + 1e-6)
    assert a[1] == 2.0 / (0.5 + 1e-6) and a[2] == a[1]          # order of the two scales does not matter
    assert a[3] == 3.0 / 1e-6
    bad = S.aspect(np.array([[np.nan, 1.0], [1.0, np.inf], [-np.inf, 1.0]], np.float32))
    assert np.all(np.isnan(bad))                                   # non-finite scales


def test_threshold_is_the_99th_percentile_of_finite_aspects():
    rng = np.random.default_rng(6)
    s = np.exp(rng.standard_normal((5000, 2))).astype(np.float32)
    a = S.aspect(s)
    ref = float(np.percentile(a, 99.0))
    assert abs(S.needle_threshold(s) - ref) <= 4 * np.spacing(ref)
    s2 = np.concatenate([s, np.array([[np.nan, 1.0]], np.float32)])
    assert S.needle_threshold(s2) == S.needle_threshold(s)
    with pytest.raises(ValueError):
        S.needle_threshold(np.full((3, 2), np.nan, np.float32))


def test_cull_removes_exactly_the_top_percent_of_distinct_aspects():
    # aspects 1 .. 1001 (distinct): position 0.99 * 1000 = 990 -> tau = 991 exactly;
    # the ten largest (992 .. 1001) are culled
    k = np.arange(1, 1002, dtype=np.float64)
    s = np.stack([k * (1.0 + 1e-6), np.ones_like(k)], 1).astype(np.float32)
    a = S.aspect(s)
    order = np.argsort(a)
    tau = S.needle_threshold(s)
    assert tau == a[order[990]]
    labels = np.ones(len(k), np.uint8)
    out, t2, n_cut = S.needle_cull(labels, s)
    assert t2 == tau and n_cut == 10
    assert np.array_equal(np.sort(np.flatnonzero(out == 0)), np.sort(order[991:]))


def test_cull_only_turns_labels_off():
    rng = np.random.default_rng(2)
    s = np.exp(rng.standard_normal((300, 2)) * 2).astype(np.float32)
    labels = (rng.random(300) < 0.5).astype(np.uint8)
    out, tau, n_cut = S.needle_cull(labels, s)
    assert np.all(out <= labels)
    assert np.array_equal(out, labels & (S.aspect(s) <= tau).astype(np.uint8))
    assert n_cut == int((S.aspect(s) > tau).sum())
