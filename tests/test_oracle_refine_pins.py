"""Pins of the mask-refinement oracle (Eq. depthband, Eq. gs-bandpass,
Eq. nerf-depthweight) against closed forms and numpy's percentile.  CPU only."""
import numpy as np
import pytest

from oracle import mask_refine as R


def _map():
    """10 x 10 median-depth map: values 1.0 .. 3.0 except the top three at 4.0,
    one pixel without a surface (0) and one NaN."""
    d = np.linspace(1.0, 3.0, 100).astype(np.float32)
    d[-3:] = 4.0
    d[10] = 0.0
    d[20] = np.nan
    return d.reshape(10, 10)


def test_depth_band_uses_prompts_and_centre_with_a_surface():
    d = np.full((8, 12), 5.0, np.float32)
    d[4, 6] = 2.5            # the centre pixel (12 // 2, 8 // 2)
    d[1, 1] = 2.0
    d[2, 9] = 3.0
    d[7, 0] = 0.0            # a prompt without a surface is left out
    assert R.depth_band(d, [(1, 1), (9, 2), (0, 7)]) == (2.0, 3.0)
    assert R.depth_band(d, []) == (2.5, 2.5)
    d[4, 6] = 0.0
    with pytest.raises(ValueError):
        R.depth_band(d, [(0, 7)])
    with pytest.raises(ValueError):
        R.depth_band(d, [(12, 0)])


def test_far_depth_is_the_98th_percentile_of_surface_pixels():
    d = np.arange(1, 101, dtype=np.float32).reshape(10, 10)
    # order statistics 98 and 99 at position 0.98 * 99 = 97.02
    pos = 0.98 * 99
    assert R.far_depth(d) == 98.0 + (99.0 - 98.0) * (pos - 97)
    rng = np.random.default_rng(4)
    m = (rng.random((37, 53)) * 9).astype(np.float32)
    m[m < 0.5] = 0.0                       # no surface
    ref = float(np.percentile(m[m > 0].astype(np.float64), 98.0))
    assert abs(R.far_depth(m) - ref) <= 4 * np.spacing(ref)
    assert R.far_depth(_map()) == 4.0      # ranks 95 and 96 of the 98 surface pixels are 4.0


def test_bandpass_closed_form_weights():
    d = _map()
    mask = np.full(d.shape, 0.75, np.float32)
    # band [2, 2] from a prompt at a pixel of depth 2 (and the centre)
    d[5, 5] = 2.0
    d[0, 0] = 2.0
    d[0, 1] = 3.0      # halfway between d_max = 2 and d_far = 4: weight 1/2
    d[0, 2] = 1.0      # nearer than the band by 1: weight 1/2
    d[0, 3] = 4.0      # at d_far: weight 0
    d[0, 4] = 9.0      # beyond d_far: clipped to 0
    out, st = R.refine_bandpass(mask, d, [(0, 0)])
    assert (st["band_min"], st["band_max"], st["d_far"]) == (2.0, 2.0, 4.0)
    assert out[0, 0] == 0.75 and out[5, 5] == 0.75
    assert out[0, 1] == np.float32(0.375) and out[0, 2] == np.float32(0.375)
    assert out[0, 3] == 0.0 and out[0, 4] == 0.0
    assert out.flat[10] == 0.0 and out.flat[20] == 0.0      # no surface, NaN
    assert out.dtype == np.float32


def test_bandpass_floor_when_the_band_reaches_d_far():
    d = np.full((4, 4), 2.0, np.float32)
    d[0, 0] = 1.0
    mask = np.ones((4, 4), np.float32)
    out, st = R.refine_bandpass(mask, d, [(1, 1)])
    assert st["d_far"] == 2.0 and st["band_max"] == 2.0   # denominator floored at 1e-6
    assert out[0, 0] == 0.0                              # 1 / 1e-6, clipped to 1
    assert np.all(out.flat[1:] == 1.0)


def test_minmax_closed_form_and_constant_depth():
    d = np.array([[1.0, 2.0, 3.0, 0.0]], np.float32)
    mask = np.array([[0.5, 0.5, 0.5, 0.5]], np.float32)
    out, st = R.refine_minmax(mask, d)
    assert (st["z_min"], st["z_max"]) == (1.0, 3.0)
    assert list(out[0]) == [0.5, 0.25, 0.0, 0.0]
    out2, _ = R.refine_minmax(mask, np.array([[2.0, 2.0, 0.0, 2.0]], np.float32))
    assert list(out2[0]) == [0.5, 0.5, 0.0, 0.5]
    with pytest.raises(ValueError):
        R.refine_minmax(mask, np.zeros((1, 4), np.float32))


def test_refined_mask_is_the_rounded_binary64_product():
    rng = np.random.default_rng(8)
    d = (1 + rng.random((16, 16)) * 3).astype(np.float32)
    m = rng.random((16, 16)).astype(np.float32)
    out, st = R.refine_bandpass(m, d, [(3, 4), (10, 12)])
    lo, hi, far = st["band_min"], st["band_max"], st["d_far"]
    for (y, x) in [(0, 0), (7, 3), (15, 15), (4, 3)]:
        D = float(d[y, x])
        band = min(max((max(lo - D, 0.0) + max(D - hi, 0.0)) / max(far - hi, 1e-6), 0.0), 1.0)
        assert out[y, x] == np.float32(float(m[y, x]) * (1.0 - band))
