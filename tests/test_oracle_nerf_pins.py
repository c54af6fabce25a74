"""Pins of the oracle's NeRF thick path (Alg. nerf-fusion; Eqs. distance_cond,
dist_tol, depth_tol, nerf-accept, nerf-vote) on exact on-axis geometry: the
voxel centre lies on the ray through its pixel's centre, so every distance is
a dyadic number and every expected value a closed form.  CPU only."""
import json
import math
import os

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


def _off_axis_case(h=H_VOX):
    """A voxel centred on the ray of pixel (399, 150), at distance t = 2 along
    it: its camera Z is t / n with n = |(199/1000, 0, 1)|."""
    cam = _cam()
    px = 399
    dx = (px + 0.5 - cam["cx"]) / cam["fx"]
    n = math.sqrt(dx * dx + 1.0)
    t = 2.0
    ctr = np.array([t * dx / n, 0.0, t / n])
    grid = dict(origin=ctr - 1.5 * h, voxel=h, dim=4)
    act = np.array([1 + 4 * (1 + 4 * 1)], np.uint32)
    return cam, grid, act, t, t / n


def _flat(cam, m, lo, mid, hi):
    full = lambda x: np.full((300, 400), x, np.float32)
    return View(cam=cam, d_cam=100.0, mask=full(m), dmin=full(lo), dmed=full(mid), dmax=full(hi), nsamp=None)


def test_planar_reading_clamps_the_ray_parameter_into_the_planar_band():
    """Default reading (the paper: both renderers report camera Z): the tuple
    is planar and x_d is the camera Z, so a planar band [z - h, z + h] around
    the voxel's camera Z passes the depth test, while t_proj = t (a ray
    distance) exceeds z + h and is clamped to D_max = z + h: delta = t - z - h
    (about 1.46h).  Without band slack (lambda = 0) the spatial gate rejects;
    with lambda = 1/2 (tau = 2h) the view votes with r = 1, w = exp(-1)."""
    cam, grid, act, t, z = _off_axis_case()
    h = H_VOX
    assert 1.2 * h < t - z - h < 1.8 * h
    v = _flat(cam, 0.9, z - h, z, z + h)
    p0 = oracle.nerf_default_params(h, "360", gamma=1.0, lambda_range=0.0)
    assert oracle.fuse(act, grid, [v], p0, variant="nerf")["vraw"][0] == 0
    p1 = oracle.nerf_default_params(h, "360", gamma=1.0, lambda_range=0.5)
    r = oracle.fuse(act, grid, [v], p1, variant="nerf")
    assert r["vraw"][0] == 1
    assert math.isclose(r["W"][0], float(np.float32(0.9)) * math.exp(-1.0), rel_tol=1e-6)
    # the same planar band read as ray distances puts the surface t - z (about
    # 2.5h) in front of the voxel along its ray: the depth test rejects
    pr = oracle.nerf_default_params(h, "360", gamma=1.0, lambda_range=0.5, nerf_ray_depths=True)
    assert oracle.fuse(act, grid, [v], pr, variant="nerf")["vraw"][0] == 0


def test_ray_reading_measures_along_the_ray():
    """Optional reading: the tuple holds distances along the pixel ray and
    x_d = t_proj.  A band [t - h, t + h] contains t_proj: delta = 0, w = 1.
    Read as planar, the same band sits t - z (about 2.5h) behind the voxel's
    camera Z and the depth test (gamma h = h) rejects."""
    cam, grid, act, t, z = _off_axis_case()
    h = H_VOX
    v = _flat(cam, 0.9, t - h, t, t + h)
    pr = oracle.nerf_default_params(h, "360", gamma=1.0, lambda_range=0.0, nerf_ray_depths=True)
    r = oracle.fuse(act, grid, [v], pr, variant="nerf")
    assert r["vraw"][0] == 1 and r["W"][0] == float(np.float32(0.9))
    pp = oracle.nerf_default_params(h, "360", gamma=1.0, lambda_range=0.0)
    assert t - z > 2.0 * h
    assert oracle.fuse(act, grid, [v], pp, variant="nerf")["vraw"][0] == 0
    # the 2DGS path on the same planes (planar, converted to ray space) rejects too
    pg = oracle.default_params(h, mask_gate=0.5)
    assert oracle.fuse(act, grid, [v], pg)["vraw"][0] == 0


def test_sample_bonus_scales_with_n_samp():
    """|x_d - d_exp| = 1.75h with gamma = 1 and b_max = 10 (no cap): n_samp = 4
    gives b = 0.8 (tau = 1.8h, accepted), n_samp = 3 gives b = 0.6 (tau = 1.6h,
    rejected), n_samp = 0 rejects; with beta = 0.1, n_samp = 8 accepts and
    n_samp = 7 rejects (the bonus is beta n_samp, linear in both)."""
    band = _band(-1.0, 1.75, 2.0)
    assert _fuse([_view(0.8, *band, nsamp=4)], use_nsamp=True, b_max=10.0)["vraw"][0] == 1
    assert _fuse([_view(0.8, *band, nsamp=3)], use_nsamp=True, b_max=10.0)["vraw"][0] == 0
    assert _fuse([_view(0.8, *band, nsamp=0)], use_nsamp=True, b_max=10.0)["vraw"][0] == 0
    assert _fuse([_view(0.8, *band, nsamp=8)], use_nsamp=True, b_max=10.0, beta=0.1)["vraw"][0] == 1
    assert _fuse([_view(0.8, *band, nsamp=7)], use_nsamp=True, b_max=10.0, beta=0.1)["vraw"][0] == 0


def test_nerf_table_thin_constants():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "nerf_hyperparams.json")))
    for col in ("llff", "360"):
        p = oracle.nerf_default_params(0.01, col)
        for k, v in g[col].items():
            assert p[k] == v, (col, k)


# ------------------------------------------------------------ NeRF thin path
# A voxel of edge 1/8 centred on the optical axis at z = 2, seen by a 200 x 160
# camera with f = 200 and the principal point at the centre of pixel (100, 80):
# its footprint is the 13 x 13 box [94, 106] x [74, 86] (closed form below).
TH = 0.125


def _thin_cam():
    c2w = np.zeros((3, 4))
    c2w[:, :3] = np.eye(3)
    return dict(fx=200.0, fy=200.0, cx=100.5, cy=80.5, c2w=c2w, width=200, height=160)


def _thin_footprint():
    cam = _thin_cam()
    us, vs = [], []
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                x, y, z = sx * TH / 2, sy * TH / 2, Z0 + sz * TH / 2
                us.append(cam["fx"] * x / z + cam["cx"])
                vs.append(cam["fy"] * y / z + cam["cy"])
    return math.floor(min(us)), math.floor(max(us)), math.floor(min(vs)), math.floor(max(vs))


def _thin_view(mask_fn=None, dexp=Z0, nsamp=None, centre_m=0.3):
    full = lambda x: np.full((160, 200), x, np.float32)
    m = full(0.9)
    if mask_fn is not None:
        m = mask_fn(m)
    m[80, 100] = centre_m                 # the centre pixel fails the thick gate
    d = full(dexp)
    ns = None if nsamp is None else np.full((160, 200), nsamp, np.uint16)
    return View(cam=_thin_cam(), d_cam=100.0, mask=m, dmin=d - 0.5 * TH, dmed=d, dmax=d + 0.5 * TH, nsamp=ns)


def _thin_fuse(views, rho=50.0, use_nsamp=False, **kw):
    ctr = np.array([0.0, 0.0, Z0])
    grid = dict(origin=ctr - 1.5 * TH, voxel=TH, dim=4)
    act = np.array([1 + 4 * (1 + 4 * 1)], np.uint32)
    p = oracle.nerf_default_params(TH, "360", **kw)
    return oracle.fuse(act, grid, views, p, use_nsamp=use_nsamp, variant="nerf", thin_rho=np.array([rho]))


def test_thin_footprint_closed_form():
    assert _thin_footprint() == (94, 106, 74, 86)


def test_nerf_thin_vote_and_eligibility():
    """Every footprint pixel but the centre is supportive (M~ 0.9, D_exp at the
    voxel): coverage 168/169 >= 0.3 and the score is the peak M~, added as
    0.9 / 1.  The thick path rejects (centre M~ 0.3).  Eligibility: the centre
    M~ must exceed 0.1 and the density reach rho_thin (30 in the 360 column)."""
    r = _thin_fuse([_thin_view()])
    assert r["vraw"][0] == 1 and r["W"][0] == float(np.float32(0.9)) and r["Z"][0] == 1.0
    assert _thin_fuse([_thin_view(centre_m=0.099)])["vraw"][0] == 0
    assert _thin_fuse([_thin_view(centre_m=0.101)])["vraw"][0] == 1
    assert _thin_fuse([_thin_view()], rho=30.0)["vraw"][0] == 1
    assert _thin_fuse([_thin_view()], rho=29.9)["vraw"][0] == 0
    # without the thin path the view casts no vote
    ctr = np.array([0.0, 0.0, Z0])
    grid = dict(origin=ctr - 1.5 * TH, voxel=TH, dim=4)
    p = oracle.nerf_default_params(TH, "360")
    assert oracle.fuse(np.array([21], np.uint32), grid, [_thin_view()], p, variant="nerf")["vraw"][0] == 0


def test_nerf_thin_doubled_multiplier_and_bonus():
    """Eq. nerf-thindepth: tau = (2 gamma + b) h.  With gamma = 0.5 (360
    column) a flat D_exp 0.75h behind the voxel is supportive (tau = h) and
    would not be with gamma h; D_exp 1.25h behind needs the bonus: n_samp = 2
    gives b = 0.4 (tau = 1.4h), n_samp = 1 gives 1.2h."""
    assert _thin_fuse([_thin_view(dexp=Z0 + 0.75 * TH)])["vraw"][0] == 1
    assert _thin_fuse([_thin_view(dexp=Z0 + 1.25 * TH)])["vraw"][0] == 0
    assert _thin_fuse([_thin_view(dexp=Z0 + 1.25 * TH, nsamp=2)], use_nsamp=True)["vraw"][0] == 1
    assert _thin_fuse([_thin_view(dexp=Z0 + 1.25 * TH, nsamp=1)], use_nsamp=True)["vraw"][0] == 0


def _first_k_pixels(k, value=0.9):
    x0, x1, y0, y1 = _thin_footprint()
    def f(m):
        m = np.full_like(m, 0.05)
        idx = [(y, x) for y in range(y0, y1 + 1) for x in range(x0, x1 + 1) if (y, x) != (80, 100)]
        for (y, x) in idx[:k]:
            m[y, x] = value
        return m
    return f


@pytest.mark.parametrize("k,votes", [(47, 0), (50, 0), (51, 1)])
def test_nerf_thin_coverage_over_all_footprint_pixels(k, votes):
    """Eq. nerf-coverage: the supportive fraction is taken over N_pixels =
    (x_end - x_start + 1)(y_end - y_start + 1) = 169: 50 supportive pixels give
    0.296 < 0.3, 51 give 0.302.  (Over a 12 x 12 = 144 box, 47 would already
    pass.)"""
    assert _thin_fuse([_thin_view(mask_fn=_first_k_pixels(k))])["vraw"][0] == votes


def test_nerf_thin_peak_is_over_every_footprint_pixel():
    """Eq. nerf-counters: m_max is the largest M~ anywhere in the footprint, not
    only among supportive pixels.  A corner pixel with M~ 0.95 whose D_exp is
    far from the voxel is not supportive but sets the score."""
    x0, x1, y0, y1 = _thin_footprint()
    v = _thin_view()
    v.mask[y0, x0] = 0.95
    v.dmed[y0, x0] = Z0 + 10 * TH
    r = _thin_fuse([v])
    assert r["vraw"][0] == 1 and r["W"][0] == float(np.float32(0.95))
