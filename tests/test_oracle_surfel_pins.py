"""Pins of the needle cull oracle (Eq. aspect, Eq. needle, Eq. pass-needle)
against closed forms, numpy's percentile and counting.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import surfel_map as S
from scenes import View


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


# ------------------------------------------------------------------ Pass 3
# Surfels seen by an identity camera (x right, y down, z forward).  The
# quaternion (w, x, y, z) = (1, 0, 0, 0) puts the tangent axes along x and y,
# so the surfel faces the camera.
def _p3_cam(W=120, H=100, f=400.0, cx=60.0, cy=50.0):
    c2w = np.zeros((3, 4))
    c2w[:, :3] = np.eye(3)
    return dict(fx=f, fy=f, cx=cx, cy=cy, c2w=c2w, width=W, height=H)


def _rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _brute_counts(cam, mask, mu, s2, q, tau_M=0.5):
    """Independent geometry: the 1-sigma box from the projected tips, then per
    pixel the ray-plane intersection X = t d with t = <mu, n> / <d, n> (camera
    at the origin), tangent coordinates u = <X - mu, r0> / s1, v = <X - mu, r1>
    / s2, accepted iff u^2 + v^2 <= 9.  Also returns the smallest distance of
    u^2 + v^2 to 9 (for the tie margin)."""
    R = _rot(q)
    mu = np.asarray(mu, np.float64)
    r0, r1 = R[:, 0], R[:, 1]
    n = np.cross(r0, r1)
    f, cx, cy = cam["fx"], cam["cx"], cam["cy"]
    proj = lambda p: (f * p[0] / p[2] + cx, f * p[1] / p[2] + cy)
    c = proj(mu)
    a0 = (np.array(proj(mu + s2[0] * r0)) - np.array(proj(mu - s2[0] * r0))) / 2
    a1 = (np.array(proj(mu + s2[1] * r1)) - np.array(proj(mu - s2[1] * r1))) / 2
    ex, ey = max(abs(a0[0]), abs(a1[0])), max(abs(a0[1]), abs(a1[1]))
    x0, x1 = max(math.floor(c[0] - ex), 0), min(math.floor(c[0] + ex), cam["width"] - 1)
    y0, y1 = max(math.floor(c[1] - ey), 0), min(math.floor(c[1] + ey), cam["height"] - 1)
    tot = hit = 0
    gap = np.inf
    for y in range(y0, y1 + 1):
        for x in range(x0, x1 + 1):
            d = np.array([(x + 0.5 - cx) / f, (y + 0.5 - cy) / f, 1.0])
            t = mu.dot(n) / d.dot(n)
            X = t * d
            u = (X - mu).dot(r0) / s2[0]
            v = (X - mu).dot(r1) / s2[1]
            rr = u * u + v * v
            gap = min(gap, abs(rr - 9.0))
            if rr <= 9.0 and X[2] > 1e-6:
                tot += 1
                hit += mask[y, x] >= tau_M
    return tot, hit, (x0, x1, y0, y1), gap


def test_face_on_surfel_counts_its_one_sigma_box():
    """A face-on isotropic surfel: the projected tangent vectors are f s / z
    along each axis, so the 1-sigma box is [c - e, c + e] with e = f s / z, and
    every pixel in it lies inside the 3-sigma disc (|u|, |v| <= 1.5 for e >= 1):
    total = the box's pixel count.  A 3-sigma box would hold about 9 times as
    many.  Mask 1 on columns < 60: mask_hit counts the box's left part."""
    cam = _p3_cam()
    mask = np.zeros((100, 120), np.float32)
    mask[:, :60] = 1.0
    mu, s = (0.013, -0.007, 2.0), 0.02
    e = 400.0 * s / 2.0
    cxp, cyp = 400.0 * mu[0] / 2.0 + 60.0, 400.0 * mu[1] / 2.0 + 50.0
    x0, x1 = math.floor(cxp - e), math.floor(cxp + e)
    y0, y1 = math.floor(cyp - e), math.floor(cyp + e)
    ok, tot, hit = oracle.surfel_view_counts(cam, mask, mu, (s, s), (1, 0, 0, 0))
    assert ok
    assert tot == (x1 - x0 + 1) * (y1 - y0 + 1)
    assert hit == (min(x1, 59) - x0 + 1) * (y1 - y0 + 1)


def test_elongated_surfel_three_sigma_test():
    """s1 = 8 s2, rotated 45 degrees in the image plane: the axis-aligned
    1-sigma box reaches 8 minor sigmas off the major axis at its anti-diagonal
    corners, which the 3-sigma test rejects.  The counts equal the brute-force
    ray-plane geometry (no pixel within 1e-6 of the u^2 + v^2 = 9 boundary)."""
    cam = _p3_cam()
    mask = (np.arange(120)[None, :] + np.arange(100)[:, None] < 110).astype(np.float32)
    mu, s2 = (0.011, 0.0037, 2.0), (0.04, 0.005)
    q = (math.cos(math.pi / 8), 0.0, 0.0, math.sin(math.pi / 8))
    ok, tot, hit = oracle.surfel_view_counts(cam, mask, mu, s2, q)
    mu32 = np.asarray(mu, np.float32).astype(np.float64)
    s32 = np.asarray(s2, np.float32).astype(np.float64)
    q32 = np.asarray(q, np.float32).astype(np.float64)
    btot, bhit, box, gap = _brute_counts(cam, mask, mu32, s32, q32)
    assert gap > 1e-6
    assert ok and (tot, hit) == (btot, bhit)
    assert 0 < tot < (box[1] - box[0] + 1) * (box[3] - box[2] + 1)      # the test rejects the corners


def test_tilted_surfels_match_ray_plane_geometry():
    """Random tilted, anisotropic surfels: Cramer's rule on the two image-plane
    conditions gives the same accepted pixels as the ray-plane intersection."""
    rng = np.random.default_rng(7)
    cam = _p3_cam()
    mask = (rng.random((100, 120)) < 0.5).astype(np.float32)
    checked = 0
    for _ in range(40):
        mu = np.array([rng.uniform(-0.1, 0.1), rng.uniform(-0.08, 0.08), rng.uniform(1.5, 3.0)], np.float32)
        s2 = rng.uniform(0.005, 0.04, 2).astype(np.float32)
        q = rng.normal(size=4).astype(np.float32)
        R = _rot(q)
        if abs(R[:, 2].dot(mu / np.linalg.norm(mu))) < 0.2:      # nearly edge-on: skip
            continue
        btot, bhit, _, gap = _brute_counts(cam, mask, mu.astype(np.float64), s2.astype(np.float64),
                                           q.astype(np.float64))
        if gap < 1e-7:
            continue
        ok, tot, hit = oracle.surfel_view_counts(cam, mask, mu, s2, q)
        assert ok and (tot, hit) == (btot, bhit)
        checked += 1
    assert checked >= 25


def test_surfel_behind_the_camera_is_not_scored():
    cam = _p3_cam()
    mask = np.ones((100, 120), np.float32)
    ok, tot, hit = oracle.surfel_view_counts(cam, mask, (0.0, 0.0, -2.0), (0.02, 0.02), (1, 0, 0, 0))
    assert not ok
    # a tip behind the camera: the surfel straddles the camera plane
    qy = (math.cos(math.pi / 4), math.sin(math.pi / 4), 0.0, 0.0)   # tangent axis 1 along z
    ok, *_ = oracle.surfel_view_counts(cam, mask, (0.0, 0.0, 0.01), (0.005, 0.05), qy)
    assert not ok


def _p3_scene():
    """Two face-on surfels in voxels 0 and 1 of a 2^3 grid of edge 1 at z in
    [1.5, 3.5); two views of the same camera whose masks cover different
    fractions of the first surfel's box."""
    cam = _p3_cam()
    grid = dict(origin=np.array([-1.0, -1.0, 1.5]), voxel=1.0, dim=2)
    xyz = np.array([[-0.05, -0.02, 2.0], [0.1, -0.02, 2.0]], np.float32)
    scales = np.full((2, 2), 0.02, np.float32)
    quats = np.tile(np.array([1, 0, 0, 0], np.float32), (2, 1))
    act = np.array([0, 1], np.uint32)          # voxels (0,0,0) and (1,0,0)
    return cam, grid, xyz, scales, quats, act


def _mask_cols(cam, frac_cols):
    """Mask 1 on the first `frac_cols` columns of surfel 0's box."""
    mu, s = (-0.05, -0.02, 2.0), 0.02
    e = cam["fx"] * s / mu[2]
    cxp = cam["fx"] * mu[0] / mu[2] + cam["cx"]
    x0 = math.floor(cxp - e)
    m = np.zeros((cam["height"], cam["width"]), np.float32)
    m[:, x0:x0 + frac_cols] = 1.0
    return m, math.floor(cxp + e) - x0 + 1


def test_kappa_is_the_max_over_gated_views_and_thresholds():
    cam, grid, xyz, scales, quats, act = _p3_scene()
    mA, ncol = _mask_cols(cam, 3)
    mB, _ = _mask_cols(cam, 6)
    assert ncol == 9
    views = [View(cam=cam, d_cam=10.0, mask=m, dmin=np.zeros_like(m), dmed=np.zeros_like(m), dmax=np.zeros_like(m))
             for m in (mA, mB)]
    labels = np.array([1, 1], np.uint8)
    # both views voted for voxel 0: kappa = max(3/9, 6/9)
    k, lab = oracle.surfel_coverage(xyz, scales, quats, labels, grid, act, np.array([3, 3], np.uint64), views)
    assert k[0] == 6.0 / 9.0 and lab[0] == 1
    # only view 0 voted (view gating): kappa = 3/9 < 0.5, culled
    k, lab = oracle.surfel_coverage(xyz, scales, quats, labels, grid, act, np.array([1, 3], np.uint64), views)
    assert k[0] == 3.0 / 9.0 and lab[0] == 0
    # no view: kappa 0
    k, lab = oracle.surfel_coverage(xyz, scales, quats, labels, grid, act, np.array([0, 3], np.uint64), views)
    assert k[0] == 0.0 and lab[0] == 0
    # surfel 1's box lies where both masks are 0
    assert k[1] == 0.0 and lab[1] == 0
    # tau_kappa is inclusive; a Pass 2 label of 0 stays 0 and is not scored
    k, lab = oracle.surfel_coverage(xyz, scales, quats, labels, grid, act, np.array([3, 3], np.uint64), views,
                                    tau_kappa=6.0 / 9.0)
    assert lab[0] == 1
    k, lab = oracle.surfel_coverage(xyz, scales, quats, np.array([0, 1], np.uint8), grid, act,
                                    np.array([3, 3], np.uint64), views)
    assert k[0] == 0.0 and lab[0] == 0


def test_mask_threshold_is_inclusive():
    cam = _p3_cam()
    for val, want in ((0.5, True), (np.nextafter(np.float32(0.5), np.float32(0)), False)):
        mask = np.full((100, 120), val, np.float32)
        ok, tot, hit = oracle.surfel_view_counts(cam, mask, (0.0, 0.0, 2.0), (0.02, 0.02), (1, 0, 0, 0))
        assert ok and tot > 0 and (hit == tot) == want and (hit == 0) != want


def test_surfel_outside_any_active_voxel_has_no_views():
    cam, grid, xyz, scales, quats, act = _p3_scene()
    m, _ = _mask_cols(cam, 9)
    views = [View(cam=cam, d_cam=10.0, mask=m, dmin=m, dmed=m, dmax=m)]
    k, lab = oracle.surfel_coverage(xyz, scales, quats, np.array([1, 1], np.uint8), grid, act[1:],
                                    np.array([1], np.uint64), views)
    assert k[0] == 0.0 and lab[0] == 0
