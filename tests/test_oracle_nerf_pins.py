"""Pins of the oracle's NeRF thick path (Alg. nerf-fusion; Eqs. distance_cond,
dist_tol, depth_tol, nerf-accept, nerf-vote) on exact on-axis geometry: the
voxel centre lies on the ray through its pixel's centre, so every distance is
a dyadic number and every expected value a closed form.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from scenes import View

H_VOX = 1.0 / 64          # dyadic voxel edge: all depths below are exact in float32
Z0 = 2.0


def _cam():
    # the centre of pixel (200, 150) is the principal point: its ray is +z
    c2w = np.zeros((3, 4))
    c2w[:, :3] = np.eye(3)
    return dict(fx=1000.0, fy=1000.0, cx=200.5, cy=150.5, c2w=c2w, width=400, height=300)


def _view(m, dmin, dexp, dmax, nsamp=None):
    cam = _cam()
    full = lambda x: np.full((300, 400), x, np.float32)
    ns = None if nsamp is None else np.full((300, 400), nsamp, np.uint16)
    return View(cam=cam, d_cam=100.0, mask=full(m), dmin=full(dmin), dmed=full(dexp), dmax=full(dmax), nsamp=ns)


def _grid():
    ctr = np.array([0.0, 0.0, Z0])
    origin = ctr - 1.5 * H_VOX
    return dict(origin=origin, voxel=H_VOX, dim=4), np.array([1 + 4 * (1 + 4 * 1)], np.uint32)


def _fuse(views, use_nsamp=False, **kw):
    grid, act = _grid()
    p = oracle.nerf_default_params(H_VOX, "360", gamma=1.0, mask_gate=0.5, **kw)
    return oracle.fuse(act, grid, views, p, use_nsamp=use_nsamp, variant="nerf")


def _band(lo, exp_, hi):
    return Z0 + lo * H_VOX, Z0 + exp_ * H_VOX, Z0 + hi * H_VOX


def test_defaults_follow_the_nerf_table():
    p = oracle.nerf_default_params(0.01, "llff")
    assert (p["gamma"], p["beta"], p["b_max"], p["lambda_range"]) == (4.0, 0.2, 10.0, 0.05)
    p = oracle.nerf_default_params(0.01, "360")
    assert (p["gamma"], p["beta"], p["b_max"], p["lambda_range"]) == (0.5, 0.2, 1.0, 5.0)


@pytest.mark.parametrize("alpha1", [1.0, 2.5])
def test_weight_inside_the_band(alpha1):
    """Band [z0 - h/2, z0 + 2h]: the voxel is inside, t_c = z0, midpoint
    z0 + 0.75h, half-width 1.25h: r = 0.6, w = exp(-0.36 alpha1)."""
    r = _fuse([_view(0.75, *_band(-0.5, 0.8, 2.0)), _view(0.9, *_band(-1.0, 0.0, 1.0))], alpha1=alpha1)
    assert r["vraw"][0] == 3
    w = math.exp(-alpha1 * 0.36)
    m1, m2 = float(np.float32(0.75)), float(np.float32(0.9))
    assert math.isclose(r["P"][0], (m1 * w + m2 * 1.0) / (w + 1.0), rel_tol=1e-12)


def test_band_slack_admits_a_voxel_in_front_of_the_band():
    """Band [z0 + 2h, z0 + 4h]: t_c = z0 + 2h, delta = 2h; tau_spatial =
    h + lambda 2h, so the vote needs lambda >= 0.5; d_exp = z0 + 0.5h keeps the
    depth test.  The weight is exp(-alpha1) (r = 1)."""
    band = _band(2.0, 0.5, 4.0)
    assert _fuse([_view(0.8, *band)], lambda_range=0.25)["vraw"][0] == 0
    assert _fuse([_view(0.8, *band)], lambda_range=0.49)["vraw"][0] == 0
    r = _fuse([_view(0.8, *band)], lambda_range=0.5)
    assert r["vraw"][0] == 1 and r["P"][0] == float(np.float32(0.8))
    assert r["W"][0] == float(np.float32(0.8)) * math.exp(-1.0)


def test_depth_tolerance_bonus_and_cap():
    """|x_d - d_exp| = 1.5h: rejected at gamma = 1 without samples; n_samp = 5
    and beta = 0.2 give b = min(1, b_max): accepted with b_max = 1
    (tau = 2h), rejected with b_max = 0.25 (tau = 1.25h)."""
    band = _band(-1.0, 1.5, 2.0)
    assert _fuse([_view(0.8, *band)])["vraw"][0] == 0
    assert _fuse([_view(0.8, *band, nsamp=5)], use_nsamp=True, b_max=1.0)["vraw"][0] == 1
    assert _fuse([_view(0.8, *band, nsamp=5)], use_nsamp=True, b_max=0.25)["vraw"][0] == 0
    assert _fuse([_view(0.8, *band, nsamp=2)], use_nsamp=True, b_max=1.0)["vraw"][0] == 0   # tau = 1.4h


def test_gates_mask_surface_and_frustum():
    band = _band(-1.0, 0.0, 1.0)
    assert _fuse([_view(0.49, *band)])["vraw"][0] == 0           # mask gate m >= 0.5
    assert _fuse([_view(0.5, *band)])["vraw"][0] == 1
    assert _fuse([_view(0.9, 0.0, 0.0, 0.0)])["vraw"][0] == 0    # no surface
    grid, act = _grid()
    v = _view(0.9, *band)
    v.cam = dict(v.cam, c2w=np.concatenate([np.diag([1.0, 1.0, -1.0]) @ np.eye(3), np.zeros((3, 1))], 1))
    p = oracle.nerf_default_params(H_VOX, "360", gamma=1.0)
    assert oracle.fuse(act, grid, [v], p, variant="nerf")["vraw"][0] == 0   # behind the camera


def test_nerf_depths_are_along_the_ray_not_planar():
    """An off-axis voxel: its ray distance exceeds its camera Z.  A band at the
    ray distance votes under NeRF; the same band read as planar depths (the
    2DGS path) puts the surface too far and the voxel fails the depth test."""
    cam = _cam()
    h = H_VOX
    # voxel centred on the ray of pixel (399, 150): direction (199, 0, 1000) / norm
    px = 399
    dx = (px + 0.5 - cam["cx"]) / cam["fx"]
    n = math.sqrt(dx * dx + 1.0)
    t = 2.0
    ctr = np.array([t * dx / n, 0.0, t / n])
    origin = ctr - 1.5 * h
    grid = dict(origin=origin, voxel=h, dim=4)
    act = np.array([1 + 4 * (1 + 4 * 1)], np.uint32)
    full = lambda x: np.full((300, 400), x, np.float32)
    v = View(cam=cam, d_cam=100.0, mask=full(0.9), dmin=full(t - h), dmed=full(t), dmax=full(t + h), nsamp=None)
    pn = oracle.nerf_default_params(h, "360", gamma=1.0, lambda_range=0.0)
    assert oracle.fuse(act, grid, [v], pn, variant="nerf")["vraw"][0] == 1
    pg = oracle.default_params(h, mask_gate=0.5)
    assert t - t / n > 1.5 * h                                      # planar vs ray gap well beyond the gates
    assert oracle.fuse(act, grid, [v], pg)["vraw"][0] == 0
