"""Pins of the oracle's thin-structure path (Alg. gs-thin, Eq. behind-gate,
Eqs. thin-nmin, gs-coverage, thin-d2min, thin-tthin-gs) on a voxel seen head-on
with a footprint of about 13 x 13 pixels, flat depth maps and a mask that
fails the thick entry gate at the centre pixel.  CPU only."""
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


def _fuse(views, rho=50.0, **kw):
    ctr = np.array([0.0, 0.0, Z0])
    grid = dict(origin=ctr - 1.5 * H, voxel=H, dim=4)
    act = np.array([1 + 4 * (1 + 4 * 1)], np.uint32)
    p = oracle.default_params(H, **kw)
    return oracle.fuse(act, grid, views, p, thin_rho=np.array([rho]))


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
    assert _fuse([_view(Z0)], rho=30.0)["vraw"][0] == 1
    assert _fuse([_view(Z0)], rho=29.99)["vraw"][0] == 0


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
