"""Pins of the oracle's thin-structure path (Alg. gs-thin, Eq. behind-gate,
Eqs. thin-nmin, gs-coverage, thin-d2min, thin-tthin-gs) on a voxel seen head-on
with a footprint of about 13 x 13 pixels, flat depth maps and a mask that
fails the thick entry gate at the centre pixel.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from scenes import View

H = 0.125
Z0 = 2.0


def _cam(f=200.0):
    c2w = np.zeros((3, 4))
    c2w[:, :3] = np.eye(3)
    return dict(fx=f, fy=f, cx=100.5, cy=80.5, c2w=c2w, width=200, height=160)


def _view(depth, f=200.0, mask_fn=None, d_cam=100.0):
    cam = _cam(f)
    m = np.full((160, 200), 0.9, np.float32)
    if mask_fn is not None:
        m = mask_fn(m)
    m[80, 100] = 0.3                      # the centre pixel fails the thick entry gate
    d = np.full((160, 200), depth, np.float32)
    return View(cam=cam, d_cam=d_cam, mask=m, dmin=d, dmed=d.copy(), dmax=d.copy(), nsamp=None)


def _fuse(views, rho=50.0, use_nsamp=False, **kw):
    ctr = np.array([0.0, 0.0, Z0])
    grid = dict(origin=ctr - 1.5 * H, voxel=H, dim=4)
    act = np.array([1 + 4 * (1 + 4 * 1)], np.uint32)
    p = oracle.default_params(H, **kw)
    return oracle.fuse(act, grid, views, p, thin_rho=np.array([rho]), use_nsamp=use_nsamp)


def test_thin_vote_is_the_peak_confidence():
    r = _fuse([_view(Z0)])
    assert r["vraw"][0] == 1
    assert r["W"][0] == float(np.float32(0.9)) and r["Z"][0] == 1.0
    assert r["P"][0] == float(np.float32(0.9))
    # without the fallback the same view casts no vote
    p = oracle.default_params(H)
    ctr = np.array([0.0, 0.0, Z0])
    plain = oracle.fuse(np.array([21], np.uint32), dict(origin=ctr - 1.5 * H, voxel=H, dim=4), [_view(Z0)], p)
    assert plain["vraw"][0] == 0


def test_density_floor():
    """The paper keeps no separate thin floor for 2DGS: the default is the
    thick path's rho_thresh = 0.5.  A larger floor is a parameter."""
    assert _fuse([_view(Z0)], rho=1.0)["vraw"][0] == 1
    assert _fuse([_view(Z0)], rho=0.49)["vraw"][0] == 0
    assert _fuse([_view(Z0)], rho=30.0, rho_thin=30.0)["vraw"][0] == 1
    assert _fuse([_view(Z0)], rho=29.99, rho_thin=30.0)["vraw"][0] == 0


def test_behind_surface_gate():
    """See-through pixels (d_cam = 1) with D_med at the voxel and D_min in
    front: the far gate compares with D_min.  With gamma = 3 every footprint
    pixel passes the front-reference depth test and unprojects (at D_med) next
    to the centre either way, so the gate alone decides: D_min 1.5h in front
    keeps the voxel (2h margin), 2.5h in front culls it."""
    def view(front):
        v = _view(Z0, d_cam=1.0)
        v.dmin = np.full_like(v.dmed, Z0 - front * H)
        return v
    assert _fuse([view(1.5)], gamma=3.0)["vraw"][0] == 1
    assert _fuse([view(2.5)], gamma=3.0)["vraw"][0] == 0


def test_support_floor_needs_25_pixels():
    """f = 200: about 169 footprint pixels; f = 40: about 9, below n_abs."""
    assert _fuse([_view(Z0, f=200.0)])["vraw"][0] == 1
    assert _fuse([_view(Z0, f=40.0)])["vraw"][0] == 0


def test_coverage_ratio():
    """Mask 0.9 on a band of columns only: about 40 % of the footprint fails
    rho_cover = 0.5, about 60 % passes."""
    def band(frac):
        def f(m):
            m = np.full_like(m, 0.1)
            lo = 94
            m[:, lo:lo + int(round(13 * frac))] = 0.9
            return m
        return f
    assert _fuse([_view(Z0, mask_fn=band(0.6))])["vraw"][0] == 1
    assert _fuse([_view(Z0, mask_fn=band(0.4))])["vraw"][0] == 0


def test_distance_gate():
    """A flat surface behind the voxel (gamma = 2 keeps it depth-consistent):
    its unprojected points lie 1.4h from the centre (kept) or 1.6h (culled)."""
    assert _fuse([_view(Z0 + 1.4 * H)], gamma=2.0)["vraw"][0] == 1
    assert _fuse([_view(Z0 + 1.6 * H)], gamma=2.0)["vraw"][0] == 0


def test_thin_and_thick_votes_combine():
    """A second view votes through the thick path (mask 0.8 everywhere,
    flat band through the voxel: w = 1): P = (0.9 + 0.8) / 2."""
    cam = _cam()
    d = np.full((160, 200), Z0, np.float32)
    thick = View(cam=cam, d_cam=100.0, mask=np.full((160, 200), 0.8, np.float32), dmin=d, dmed=d.copy(),
                 dmax=d.copy(), nsamp=None)
    r = _fuse([_view(Z0), thick])
    assert r["vraw"][0] == 3
    m1, m2 = float(np.float32(0.9)), float(np.float32(0.8))
    assert r["P"][0] == pytest.approx((m1 + m2) / 2.0, rel=1e-15)


def _footprint(f):
    """Closed-form footprint of the voxel: its near face (z = Z0 - h/2) spans
    x, y in [-h/2, h/2]; pixel box floor(min)..floor(max) of the 8 corners."""
    cam = _cam(f)
    us, vs = [], []
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                z = Z0 + sz * H / 2
                us.append(f * (sx * H / 2) / z + cam["cx"])
                vs.append(f * (sy * H / 2) / z + cam["cy"])
    return math.floor(min(us)), math.floor(max(us)), math.floor(min(vs)), math.floor(max(vs))


def _surface_on(k, f):
    """A view where only k footprint pixels (the centre first, then raster
    order) have a surface at the voxel; every other pixel has none."""
    x0, x1, y0, y1 = _footprint(f)
    v = _view(Z0, f=f)
    keep = np.zeros(v.dmed.shape, bool)
    idx = [(80, 100)] + [(y, x) for y in range(y0, y1 + 1) for x in range(x0, x1 + 1) if (y, x) != (80, 100)]
    for (y, x) in idx[:k]:
        keep[y, x] = True
    for a in (v.dmin, v.dmed, v.dmax):
        a[~keep] = 0.0
    return v


def test_support_floor_is_the_ceiling_of_the_footprint_fraction():
    """Eq. thin-nmin with a footprint of more than 250 pixels, where
    ceil(rho_occ A_B) binds: f = 260 gives the 17 x 17 box, A_B = |B| = 289
    (pixels, with the +1), n_min = ceil(28.9) = 29.  29 depth-consistent pixels
    vote, 28 do not (a floor, or A_B = 16 x 16, would let 28 through)."""
    x0, x1, y0, y1 = _footprint(260.0)
    assert (x1 - x0 + 1, y1 - y0 + 1) == (17, 17)
    assert math.ceil(0.1 * 289) == 29
    assert _fuse([_surface_on(29, 260.0)])["vraw"][0] == 1
    assert _fuse([_surface_on(28, 260.0)])["vraw"][0] == 0


def test_tightening_uses_each_pixels_own_excess():
    """n_samp 12 on the even pixels ((x + y) even, 85 of the 13 x 13 footprint,
    the centre among them), 10 on the odd ones: mean 11.006, sigma 1.0, so no
    pixel is layered, and with beta = 1 the even pixels' tolerance tightens to
    h / (1 + 0.994) = 0.50h while the odd ones keep h.  The surface is 0.75h
    behind the voxel everywhere.  M~ 0.9 on the odd pixels: they alone are
    depth-consistent and mask-positive (coverage 1), 84 >= 25, the view votes.
    Without the per-pixel tightening all 169 would count and the coverage
    84/169 < 0.5 would reject; with the centre pixel's excess everywhere none
    would count."""
    x0, x1, y0, y1 = _footprint(200.0)
    yy, xx = np.mgrid[0:160, 0:200]
    even = (xx + yy) % 2 == 0
    ns = np.where(even, 12, 10).astype(np.uint16)
    v = _view(Z0 + 0.75 * H, mask_fn=lambda m: np.where(even, np.float32(0.1), np.float32(0.9)))
    v.nsamp = ns
    fp = even[y0:y1 + 1, x0:x1 + 1]
    assert fp.sum() == 85 and (~fp).sum() == 84
    S1 = int(ns[y0:y1 + 1, x0:x1 + 1].astype(np.int64).sum())
    S2 = int((ns[y0:y1 + 1, x0:x1 + 1].astype(np.int64) ** 2).sum())
    A = 169
    assert (12 * A - S1) ** 2 <= A * S2 - S1 * S1            # the 12s are not layered
    r = _fuse([v], beta=1.0, use_nsamp=True)
    assert r["vraw"][0] == 1 and r["W"][0] == float(np.float32(0.9))


def test_layered_pixels_unproject_at_the_front_hit():
    """30 footprint pixels (the centre first) carry n_samp 30 among 1s: they are
    layered (a minority far above mean + sigma), so their gate uses D_min,
    which sits at the voxel (accepted), and they unproject at D_min, next to
    the voxel centre.  D_med is 3h behind: unprojected there they would fail
    the 1.5h distance gate, and the median reference would fail the depth
    gate.  Other footprint pixels have no surface."""
    x0, x1, y0, y1 = _footprint(200.0)
    v = _surface_on(30, 200.0)
    lay = v.dmed > 0
    ns = np.where(lay, 30, 1).astype(np.uint16)
    v.nsamp = ns
    v.dmin = np.where(lay, np.float32(Z0), np.float32(0.0)).astype(np.float32)
    v.dmed = np.where(lay, np.float32(Z0 + 3 * H), np.float32(0.0)).astype(np.float32)
    v.dmax = v.dmed.copy()
    n = ns[y0:y1 + 1, x0:x1 + 1].astype(np.int64)
    S1, S2, A = int(n.sum()), int((n * n).sum()), n.size
    assert (30 * A - S1) > 0 and (30 * A - S1) ** 2 > A * S2 - S1 * S1
    r = _fuse([v], use_nsamp=True)
    assert r["vraw"][0] == 1 and r["W"][0] == float(np.float32(0.9))


def test_seethrough_pixels_use_the_front_reference():
    """d_cam = 1.4: pixels with D_med = Z0 + 1.2h (> 1.5 d_cam = Z0 + 0.8h) are
    see-through; their D_min = Z0 - 0.2h is trusted, so the one-sided gate
    on D_min accepts (0.2h), while the median would reject (1.2h > h).
    Unprojected at D_med (not layered) they lie 1.2h from the centre, inside
    the 1.5h gate: the view votes.  With D_min above D_med (untrusted) the
    front reference is not taken and the median gate rejects every pixel."""
    def view(dmin):
        v = _view(Z0 + 1.2 * H, d_cam=1.4)
        v.dmin = np.full_like(v.dmed, np.float32(dmin))
        return v
    assert _fuse([view(Z0 - 0.2 * H)])["vraw"][0] == 1
    assert _fuse([view(Z0 + 1.4 * H)])["vraw"][0] == 0
