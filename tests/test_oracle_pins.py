"""Pins of the CPU oracle against things other than itself: closed forms,
brute force, exact rational arithmetic and invariants the paper states.

A planted mistake in any oracle step (dropped term, sign, index, transposed
operand) should fail at least one of these.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes
from scenes import View

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ident_cam(W=100, H=80, f=100.0, cx=50.0, cy=40.0, o=(0.0, 0.0, 0.0), R=None):
    c2w = np.zeros((3, 4))
    c2w[:, :3] = np.eye(3) if R is None else R
    c2w[:, 3] = o
    return dict(fx=f, fy=f, cx=cx, cy=cy, c2w=c2w, width=W, height=H)


def flat_view(cam, m, dmin, dmed, dmax, d_cam=100.0, nsamp=None):
    H, W = cam["height"], cam["width"]
    full = lambda x: np.full((H, W), x, np.float32)
    return View(cam=cam, d_cam=d_cam, mask=full(m), dmin=full(dmin), dmed=full(dmed), dmax=full(dmax),
                nsamp=nsamp)


def grid_for_voxel(center, h):
    """A 4^3 grid whose voxel (1,1,1) is centred at ``center``."""
    origin = np.asarray(center, np.float64) - 1.5 * h
    return dict(origin=origin, voxel=h, dim=4), np.array([1 + 4 * (1 + 4 * 1)], np.uint32)


# ------------------------------------------------------------------ golden
def test_default_params_match_paper_table():
    g = json.load(open(os.path.join(GOLDEN, "gs_hyperparams.json")))
    p = oracle.default_params(0.01)
    for k in ("gamma", "beta", "gamma_st", "tau_cons", "mask_gate"):
        assert p[k] == g[k], k


# -------------------------------------------------------------- projection
def test_projection_identity_pose_closed_form():
    cam = ident_cam()
    ok, u, v, qz = oracle.project(cam, [0.5, -0.25, 2.0])
    assert ok and u == 100 * 0.5 / 2 + 50 and v == 100 * -0.25 / 2 + 40 and qz == 2.0
    ok, *_ = oracle.project(cam, [0.0, 0.0, -1.0])
    assert not ok
    ok, *_ = oracle.project(cam, [0.0, 0.0, 0.0])
    assert not ok


def test_projection_axis_permutation_pose():
    # camera axes: right = +y, down = +z, forward = +x (right x down = forward)
    R = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    o = np.array([1.0, 2.0, 3.0])
    cam = ident_cam(R=R, o=o)
    p = o + 2.0 * R[:, 2] + 0.5 * R[:, 0] - 0.25 * R[:, 1]
    ok, u, v, qz = oracle.project(cam, p)
    assert ok and qz == 2.0 and u == 75.0 and v == 27.5


def test_pixel_ray_and_planar_to_ray_closed_form():
    cam = ident_cam(f=80.0, cx=33.0, cy=21.0)
    for px, py in [(0, 0), (33, 21), (99, 79), (10, 60)]:
        d, cosv = oracle.pixel_ray(cam, px, py)
        r = np.array([(px + 0.5 - 33.0) / 80.0, (py + 0.5 - 21.0) / 80.0, 1.0])
        assert np.allclose(d, r / np.linalg.norm(r), rtol=0, atol=1e-15)
        # a fronto-parallel plane Z = z0: ray depth = z0 * |r|
        z0 = 2.5
        assert math.isclose(z0 / cosv, z0 * math.sqrt(r @ r), rel_tol=1e-14)


# ------------------------------------------------------------------- pi_dg
def test_pi_dg_flat_and_ramp():
    H, W = 6, 7
    d = np.full((H, W), 3.0, np.float32)
    assert np.all(oracle.pi_dg_map(d, d, k=10.0) == 1.0)
    a = 0.25
    ramp = (a * np.arange(W, dtype=np.float64))[None, :].repeat(H, 0).astype(np.float32)
    k = 2.0
    # d = (dmin + dmax)/2 with dmin = ramp, dmax = ramp + 1 -> d = ramp + 0.5
    pi = oracle.pi_dg_map(ramp, ramp + np.float32(1.0), k=k)
    assert np.allclose(pi[:, 1:-1], math.exp(-k * (2 * a) ** 2), rtol=1e-14)
    assert np.allclose(pi[:, [0, -1]], math.exp(-k * a ** 2), rtol=1e-14)


# ------------------------------------------------------- footprint statistics
def test_layered_predicate_matches_float_statistics():
    rng = np.random.default_rng(0)
    checked = 0
    for trial in range(400):
        H, W = rng.integers(2, 12, size=2)
        hi = int(rng.choice([3, 50, 65535]))
        ns = rng.integers(0, hi + 1, size=(H, W)).astype(np.uint16)
        x0, x1 = sorted(rng.integers(0, W, size=2))
        y0, y1 = sorted(rng.integers(0, H, size=2))
        n = int(rng.integers(0, hi + 1))
        lay, E = oracle.footprint_stats(ns, x0, x1, y0, y1, n)
        blk = ns[y0:y1 + 1, x0:x1 + 1].astype(np.float64)
        mean, sd = blk.mean(), blk.std()
        if abs(n - mean - sd) < 1e-6 * (1 + abs(n)):
            continue  # a near-tie is decided exactly by the integer form only
        assert lay == (n > mean + sd)
        assert math.isclose(E, max(n - mean, 0.0), rel_tol=1e-12, abs_tol=1e-12)
        checked += 1
    assert checked > 350


# ------------------------------------------------------------------ Morton
def _morton_str(x, y, z, bits=10):
    bx, by, bz = (format(t, f"0{bits}b") for t in (x, y, z))
    s = "".join(bz[i] + by[i] + bx[i] for i in range(bits))
    return int(s, 2)


def test_morton_known_codes_and_bijection():
    assert oracle.morton3(1, 0, 0) == 1 and oracle.morton3(0, 1, 0) == 2 and oracle.morton3(0, 0, 1) == 4
    assert oracle.morton3(2, 0, 0) == 8 and oracle.morton3(3, 3, 3) == 63
    g = 16
    codes = {oracle.morton3(x, y, z) for x in range(g) for y in range(g) for z in range(g)}
    assert codes == set(range(g ** 3))
    rng = np.random.default_rng(1)
    for x, y, z in rng.integers(0, 1024, size=(200, 3)):
        assert oracle.morton3(int(x), int(y), int(z)) == _morton_str(int(x), int(y), int(z))


# ------------------------------------------------------- voxel index / labels
@pytest.mark.parametrize("origin,h,dim", [((-1.0, -1.0, -1.0), 2.0 / 64, 64),
                                          ((-2.3, 0.7, 2.9), 0.0173, 128)])
def test_point_voxel_matches_exact_rational(origin, h, dim):
    rng = np.random.default_rng(2)
    grid = dict(origin=np.array(origin), voxel=h, dim=dim)
    ext = h * dim
    pts = (np.array(origin) + rng.uniform(-0.05 * ext, 1.05 * ext, size=(3000, 3))).astype(np.float32)
    pts[::97, 1] = np.nan
    flagged = 0
    for p in pts:
        got = oracle.point_voxel(p, grid)
        if np.isnan(p).any():
            assert got == -1
            continue
        idx = []
        near = False
        for k in range(3):
            q = (Fraction(float(p[k])) - Fraction(origin[k])) / Fraction(h)
            f = math.floor(q)
            near |= abs(q - round(q)) < Fraction(1, 10 ** 9)
            idx.append(f)
        inside = all(0 <= i < dim for i in idx)
        exp = idx[0] + dim * (idx[1] + dim * idx[2]) if inside else -1
        if near:
            flagged += 1
            continue
        assert got == exp
    assert flagged < 10


def test_occupancy_brute_force_with_opacity():
    rng = np.random.default_rng(3)
    grid = dict(origin=np.array([0.0, 0.0, 0.0]), voxel=0.25, dim=8)
    pts = rng.uniform(-0.2, 2.2, size=(500, 3)).astype(np.float32)
    op = rng.uniform(0, 0.4, size=500).astype(np.float32)
    tau = 0.5
    rho = {}
    for i, p in enumerate(pts):
        f = [math.floor((Fraction(float(p[k])) - 0) / Fraction(1, 4)) for k in range(3)]
        if all(0 <= t < 8 for t in f):
            lin = f[0] + 8 * (f[1] + 8 * f[2])
            rho[lin] = rho.get(lin, 0.0) + float(op[i])
    act_exp = sorted([l for l, r in rho.items() if r >= tau],
                     key=lambda l: _morton_str(l % 8, (l // 8) % 8, l // 64))
    act, r = oracle.occupancy(pts, grid, opacity=op, tau_occ=tau, with_rho=True)
    assert list(act) == act_exp
    assert np.array_equal(r, np.array([rho[l] for l in act_exp]))
    # unit opacity: integer counts, tau <= 1 -> every voxel holding a point
    act1 = oracle.occupancy(pts, grid)
    assert set(act1.tolist()) == set(rho.keys())


def test_zero_occupancy_and_empty_outputs():
    grid = dict(origin=np.zeros(3), voxel=0.1, dim=16)
    act = oracle.occupancy(np.zeros((0, 3), np.float32), grid)
    assert len(act) == 0
    cam = ident_cam()
    v = flat_view(cam, 1.0, 1.0, 1.0, 1.0)
    r = oracle.fuse(act, grid, [v], oracle.default_params(0.1))
    assert len(r["P"]) == 0 and list(r["counts"]) == [0, 0, 0]
    lab = oracle.label(np.array([[0.05, 0.05, 0.05]], np.float32), grid, act)
    assert lab.tolist() == [0]


# -------------------------------------------------------------- gates / votes
def test_out_of_frustum_no_votes():
    s = scenes.make_tiny_sphere(dim=32, n_points=3000, width=64, height=48, focal=50.0)
    act = oracle.occupancy(s.points, s.grid)
    away = []
    for v in s.views:
        cam = dict(v.cam)
        c2w = cam["c2w"].copy()
        c2w[:, 0] *= -1.0  # turn around: forward and right flip, down kept
        c2w[:, 2] *= -1.0
        cam["c2w"] = c2w
        away.append(View(cam=cam, d_cam=v.d_cam, mask=v.mask, dmin=v.dmin, dmed=v.dmed, dmax=v.dmax))
    r = oracle.fuse(act, s.grid, away, oracle.default_params(s.voxel))
    assert np.all(r["P"] == 0) and np.all(r["vraw"] == 0)


def test_wall_head_on_closed_form():
    """Identity camera, fronto-parallel wall Z = z0 with a degenerate band:
    accepted iff |c - z0 r_pix| <= h (spatial gate, pi = 1 on a flat map) and
    |c_z - z0| <= gamma h; the surface point is the ray/plane intersection."""
    h, z0, f = 0.05, 2.0, 100.0
    cam = ident_cam(W=200, H=160, f=f, cx=100.0, cy=80.0)
    v = flat_view(cam, 1.0, z0, z0, z0)
    dim = 24
    origin = np.array([-0.3, -0.3, z0 - 12 * h + 0.013])
    grid = dict(origin=origin, voxel=h, dim=dim)
    act = np.arange(dim ** 3, dtype=np.uint32)
    p = oracle.default_params(h)
    r = oracle.fuse(act, grid, [v], p)
    acc = r["vraw"] == 1
    i = act % dim
    j = (act // dim) % dim
    k = act // (dim * dim)
    c = origin + (np.stack([i, j, k], 1) + 0.5) * h
    u = f * c[:, 0] / c[:, 2] + 100.0
    vv = f * c[:, 1] / c[:, 2] + 80.0
    inframe = (u >= 0) & (u < 200) & (vv >= 0) & (vv < 160)
    px, py = np.floor(u), np.floor(vv)
    rp = np.stack([(px + 0.5 - 100.0) / f, (py + 0.5 - 80.0) / f, np.ones_like(u)], 1)
    dist = np.linalg.norm(c - z0 * rp, axis=1)
    exp = inframe & (dist <= h) & (np.abs(c[:, 2] - z0) <= p["gamma"] * h)
    slack = np.minimum(np.abs(dist - h), np.abs(np.abs(c[:, 2] - z0) - h))
    sure = slack > 1e-9
    assert exp.sum() > 20
    assert np.array_equal(acc[sure], exp[sure])
    assert np.all(r["P"][acc] == 1.0)


def _single_voxel_two_views(mA, mB, bandB, gamma_st=1.5, d_camB=100.0, mask_gate=0.0):
    h = 0.02
    cam = ident_cam(W=400, H=300, f=10000.0, cx=200.0, cy=150.0)
    ctr = np.array([0.0003, -0.0002, 2.0])
    grid, act = grid_for_voxel(ctr, h)
    c = grid["origin"] + 1.5 * h
    xd = float(c[2])
    vA = flat_view(cam, mA, xd, xd, xd)
    dminB, dmedB, dmaxB = (xd + b * h for b in bandB)
    vB = flat_view(cam, mB, dminB, dmedB, dmaxB, d_cam=d_camB)
    p = oracle.default_params(h, mask_gate=mask_gate, gamma_st=gamma_st)
    return oracle.fuse(act, grid, [vA, vB], p), h


def test_depth_weight_closed_form():
    """View A: degenerate band through the voxel -> r = 0, w = 1.  View B:
    surface band starts 0.1h behind the voxel, so t is clamped to the band's
    front and r = -1, w = exp(-alpha1).  P = (mA + mB e^-1) / (1 + e^-1)."""
    mA, mB = 0.9, 0.3
    r, _ = _single_voxel_two_views(mA, mB, (0.1, 0.3, 0.5))
    assert r["vraw"][0] == 3
    mA32, mB32 = float(np.float32(mA)), float(np.float32(mB))
    w = math.exp(-1.0)
    assert math.isclose(r["P"][0], (mA32 + mB32 * w) / (1 + w), rel_tol=1e-12)


def test_seethrough_switches_to_front_reference():
    """A pixel whose median depth exceeds gamma_ST * d_cam uses the one-sided
    gate on D_min.  Band B = [x_d - 1.5h, x_d, x_d + 1.5h]: the median test
    accepts the voxel (|0| <= h); the front test rejects it (1.5h > h)."""
    r_med, _ = _single_voxel_two_views(0.9, 0.3, (-1.5, 0.0, 1.5), d_camB=100.0)
    assert r_med["vraw"][0] == 3
    r_front, _ = _single_voxel_two_views(0.9, 0.3, (-1.5, 0.0, 1.5), d_camB=1.0)
    assert r_front["vraw"][0] == 1
    # a voxel sitting at the front of the band is accepted by the front test
    r_f2, _ = _single_voxel_two_views(0.9, 0.3, (0.0, 1.5, 3.0), d_camB=1.0)
    assert r_f2["vraw"][0] == 3
    r_m2, _ = _single_voxel_two_views(0.9, 0.3, (0.0, 1.5, 3.0), d_camB=100.0)
    assert r_m2["vraw"][0] == 1


def test_untrusted_pixel_does_not_vote():
    r, _ = _single_voxel_two_views(0.9, 0.3, (0.2, 0.0, 0.5))  # D_min > D_med
    assert r["vraw"][0] == 1


def test_mask_gate_R1_range_and_single_view_identity():
    s = scenes.make_tiny_sphere(dim=32, n_points=4000, width=64, height=48, focal=50.0)
    act = oracle.occupancy(s.points, s.grid)
    p = oracle.default_params(s.voxel)
    r = oracle.fuse(act, s.grid, s.views, p)
    P = r["P"]
    assert np.all((P == 0) | ((P >= 0.5) & (P <= 1.0)))
    # single view: the float32 P equals the mask at the projected pixel, exactly
    v = s.views[1]
    r1 = oracle.fuse(act, s.grid, [v], p)
    voted = np.flatnonzero(r1["vraw"] == 1)
    assert len(voted) > 10
    for a in voted:
        l = int(act[a])
        c = s.origin + (np.array([l % 32, (l // 32) % 32, l // 1024]) + 0.5) * s.voxel
        ok, u, vv, _ = oracle.project(v.cam, c)
        assert ok
        # (m w) / w rounds once in binary64; the float32 output is m exactly
        assert np.float32(r1["P"][a]) == v.mask[int(math.floor(vv)), int(math.floor(u))]
    # a view listed twice gives the same P, bit for bit
    r2 = oracle.fuse(act, s.grid, [v, v], p)
    assert np.array_equal(r2["P"], r1["P"])
    assert np.array_equal(r2["vraw"] != 0, r1["vraw"] != 0)


def test_degenerate_band_gives_mean_of_votes():
    s = scenes.make_tiny_sphere(dim=32, n_points=4000, width=64, height=48, focal=50.0)
    views = [View(cam=v.cam, d_cam=v.d_cam, mask=v.mask, dmin=v.dmed, dmed=v.dmed, dmax=v.dmed)
             for v in s.views]
    act = oracle.occupancy(s.points, s.grid)
    p = oracle.default_params(s.voxel, mask_gate=0.0)
    r = oracle.fuse(act, s.grid, views, p)
    multi = np.flatnonzero(np.array([bin(int(x)).count("1") for x in r["vraw"]]) >= 2)
    assert len(multi) > 10
    for a in multi[:200]:
        l = int(act[a])
        c = s.origin + (np.array([l % 32, (l // 32) % 32, l // 1024]) + 0.5) * s.voxel
        ms = []
        for si, v in enumerate(views):
            if (int(r["vraw"][a]) >> si) & 1:
                _, u, vv, _ = oracle.project(v.cam, c)
                ms.append(float(v.mask[int(math.floor(vv)), int(math.floor(u))]))
        assert math.isclose(r["P"][a], sum(ms) / len(ms), rel_tol=1e-14)


def test_consensus_mask_and_counts():
    s = scenes.make_tiny_sphere(dim=32, n_points=4000, width=64, height=48, focal=50.0)
    act = oracle.occupancy(s.points, s.grid)
    p = oracle.default_params(s.voxel, mask_gate=0.0)
    r = oracle.fuse(act, s.grid, s.views, p)
    seg = r["P"] >= 0.5
    assert np.array_equal(r["seg"].astype(bool), seg)
    assert np.array_equal(r["vout"], np.where(seg, r["vraw"], 0))
    assert r["counts"][0] == seg.sum()
    assert r["counts"][2] == sum(bin(int(x)).count("1") for x in r["vraw"])
    assert np.all(r["P"][r["vraw"] == 0] == 0)


# --------------------------------------------------------- analytic sphere
def test_analytic_sphere_precision_and_recall():
    """Noise-free hard masks of the unit sphere; pi_dg switched off (k = 0).
    Precision: a vote needs the pixel ray to hit the sphere and the voxel to lie
    within h of the segment [t_hit - h/2, t_hit] of that ray, so every
    segmented voxel is within 1.5h of the sphere.  Recall: every active voxel
    within h/4 of the sphere, front-facing to some camera with cos > 0.8, is
    segmented (fine pixels: 1/4 voxel)."""
    s = scenes.make_tiny_sphere(dim=64, n_points=40000, n_views=4, width=512, height=384, focal=400.0,
                                mask_noise=0.0, slope=1e4)
    act = oracle.occupancy(s.points, s.grid)
    p = oracle.default_params(s.voxel, k_grad=0.0)
    r = oracle.fuse(act, s.grid, s.views, p)
    h = s.voxel
    g = s.dim
    idx = np.stack([act % g, (act // g) % g, act // (g * g)], 1)
    c = s.origin + (idx + 0.5) * h
    dist = np.abs(np.linalg.norm(c, axis=1) - 1.0)
    seg = r["seg"].astype(bool)
    assert seg.sum() > 1000
    assert dist[seg].max() <= 1.5 * h + 1e-12
    nrm = c / np.linalg.norm(c, axis=1, keepdims=True)
    facing = np.zeros(len(act), bool)
    for v in s.views:
        o = v.cam["c2w"][:, 3]
        to_cam = o - c
        to_cam /= np.linalg.norm(to_cam, axis=1, keepdims=True)
        facing |= (nrm * to_cam).sum(1) > 0.8
    want = (dist <= h / 4) & facing
    assert want.sum() > 500
    assert np.all(seg[want])


# ------------------------------------------------ exact-geometry single voxel
# Identity camera with f = 8192 px, voxel edge h = 2^-6 and a voxel centre on
# the ray through the centre of pixel (201, 149): c = (3/8192, -1/8192, 2).
# Every quantity below is dyadic, so the closed forms are exact.
_H = 2.0 ** -6
_F = 8192.0


def _exact_cam():
    return ident_cam(W=400, H=300, f=_F, cx=200.0, cy=150.0)


def _exact_voxel():
    ctr = np.array([3.0 / 8192.0, -1.0 / 8192.0, 2.0])
    return grid_for_voxel(ctr, _H)


def _band(cam, m, lo, med, hi, d_cam=100.0, nsamp=None):
    return flat_view(cam, m, 2.0 + lo * _H, 2.0 + med * _H, 2.0 + hi * _H, d_cam=d_cam, nsamp=nsamp)


@pytest.mark.parametrize("alpha1", [1.0, 2.5])
def test_depth_weight_interior_closed_form(alpha1):
    """View A: degenerate band through the voxel, w = 1.  View B: band
    [x_d - h/2, x_d + 2h] (median x_d + 0.8h); the voxel lies inside the band,
    so t = <c, d> and r = (0 - 0.75h) / 1.25h = -0.6: w = exp(-alpha1 0.36)."""
    cam = _exact_cam()
    grid, act = _exact_voxel()
    vA = _band(cam, 0.75, 0.0, 0.0, 0.0)
    vB = _band(cam, 0.25, -0.5, 0.8, 2.0)
    p = oracle.default_params(_H, mask_gate=0.0, alpha1=alpha1)
    r = oracle.fuse(act, grid, [vA, vB], p)
    assert r["vraw"][0] == 3
    w = math.exp(-alpha1 * 0.36)
    assert math.isclose(r["P"][0], (0.75 + 0.25 * w) / (1 + w), rel_tol=1e-12)
    # see-through: the reference switches to D_min, t is clamped to the band
    # front, r = -1: w = exp(-alpha1)
    vBf = _band(cam, 0.25, -0.5, 0.8, 2.0, d_cam=1.0)
    r2 = oracle.fuse(act, grid, [vA, vBf], p)
    assert r2["vraw"][0] == 3
    w2 = math.exp(-alpha1)
    assert math.isclose(r2["P"][0], (0.75 + 0.25 * w2) / (1 + w2), rel_tol=1e-12)


def _footprint_area(cam, grid):
    us, vs = [], []
    o = grid["origin"]
    for j in range(8):
        p = [o[a] + (1 + ((j >> a) & 1)) * grid["voxel"] for a in range(3)]
        ok, u, v, _ = oracle.project(cam, p)
        assert ok
        us.append(u)
        vs.append(v)
    return (math.floor(max(us)) - math.floor(min(us)) + 1) * (math.floor(max(vs)) - math.floor(min(vs)) + 1)


@pytest.mark.parametrize("side", [0.97, 1.03])
def test_depth_tolerance_tightening_closed_form(side):
    """n_samp = 1 everywhere but K + 1 at the voxel's pixel: over a footprint of
    A pixels the excess is E = K (A - 1) / A and the tolerance gamma h / (1 + beta E).
    The surface sits a = side * tolerance in front of the voxel."""
    cam = _exact_cam()
    grid, act = _exact_voxel()
    K = 100
    A = _footprint_area(cam, grid)
    E = K * (A - 1) / A
    tol = _H / (1 + 0.05 * E)
    a = side * tol
    H_, W_ = cam["height"], cam["width"]
    ns = np.ones((H_, W_), np.uint16)
    ns[149, 201] = K + 1
    d = 2.0 - a
    v = flat_view(cam, 1.0, d, d, d, nsamp=ns)
    p = oracle.default_params(_H)
    with_ns = oracle.fuse(act, grid, [v], p, use_nsamp=True)
    without = oracle.fuse(act, grid, [v], p, use_nsamp=False)
    assert without["vraw"][0] == 1           # a < h: accepted without tightening
    assert with_ns["vraw"][0] == (1 if side < 1 else 0)


def test_occupancy_threshold_is_inclusive():
    grid = dict(origin=np.zeros(3), voxel=1.0, dim=4)
    pts = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5], [1.6, 0.6, 0.6], [2.5, 2.5, 2.5]], np.float32)
    op = np.array([0.5, 0.25, 0.25, 0.49], np.float32)
    act = oracle.occupancy(pts, grid, opacity=op, tau_occ=0.5)
    assert sorted(act.tolist()) == [0, 1]     # rho == tau is active; 0.49 is not
    act1 = oracle.occupancy(pts, grid, tau_occ=1.0)
    assert sorted(act1.tolist()) == [0, 1, 42]
    act2 = oracle.occupancy(pts, grid, tau_occ=2.0)
    assert act2.tolist() == [1]


@pytest.mark.parametrize("kind", ["seethrough", "layered"])
def test_front_gate_is_one_sided(kind):
    """Eq. asym-gate: with the front reference (see-through, or layered by the
    footprint statistics) the gate is x_d - D_min <= t_depth, one-sided.  The
    surface's front hit D_min lies 0.75h behind the voxel (the voxel is in
    front of it): the one-sided gate accepts, an absolute value would reject
    (t_depth = 0.5h with gamma = 0.5, or about h/6 with the excess of a layered
    pixel).  The ray through the voxel's pixel centre passes through the
    voxel centre, so t is clamped to D_min^ray and delta = 0.75h (times the
    tiny obliquity), inside tau_sp = h on flat maps; r = -1 gives w = exp(-1)."""
    cam = _exact_cam()
    grid, act = _exact_voxel()
    if kind == "seethrough":
        v = _band(cam, 0.6, 0.75, 2.0, 2.0, d_cam=1.0)
        p = oracle.default_params(_H, gamma=0.5)
        use_ns = False
    else:
        ns = np.ones((cam["height"], cam["width"]), np.uint16)
        ns[149, 201] = 101
        v = _band(cam, 0.6, 0.75, 2.0, 2.0, nsamp=ns)
        p = oracle.default_params(_H)
        use_ns = True
    r = oracle.fuse(act, grid, [v], p, use_nsamp=use_ns)
    assert r["vraw"][0] == 1
    assert math.isclose(r["W"][0], float(np.float32(0.6)) * math.exp(-1.0), rel_tol=1e-9)
    # a voxel behind D_min by more than t_depth is rejected by the same gate
    if kind == "seethrough":
        vb = _band(cam, 0.6, -0.75, 2.0, 2.0, d_cam=1.0)
        assert oracle.fuse(act, grid, [vb], p)["vraw"][0] == 0


def test_pi_dg_centre_depth_uses_both_ends_of_the_band():
    """App. D: the centre depth is (D_min + D_max) / 2.  A ramp in D_max alone
    (D_min flat) gives half the gradient of the ramp."""
    H, W = 5, 6
    a = 0.5
    dmin = np.full((H, W), 2.0, np.float32)
    dmax = (2.0 + a * np.arange(W, dtype=np.float64))[None, :].repeat(H, 0).astype(np.float32)
    k = 3.0
    pi = oracle.pi_dg_map(dmin, dmax, k=k)
    assert np.allclose(pi[:, 1:-1], math.exp(-k * a ** 2), rtol=1e-14)   # g_x = (a / 2) * 2


def test_gate_and_consensus_ties_are_inclusive():
    """A mask value exactly at the entry gate votes (m >= gate), and a voxel
    whose P equals tau_cons exactly is segmented (P >= tau_cons)."""
    cam = _exact_cam()
    grid, act = _exact_voxel()
    v = _band(cam, 0.5, 0.0, 0.0, 0.0)
    r = oracle.fuse(act, grid, [v], oracle.default_params(_H))
    assert r["vraw"][0] == 1 and r["P"][0] == 0.5
    assert r["seg"][0] == 1 and r["vout"][0] == 1 and r["counts"][0] == 1 and r["counts"][1] == 1
    below = _band(cam, float(np.nextafter(np.float32(0.5), np.float32(0.0))), 0.0, 0.0, 0.0)
    assert oracle.fuse(act, grid, [below], oracle.default_params(_H))["vraw"][0] == 0


def test_footprint_with_a_corner_behind_the_camera_has_no_statistics():
    """A voxel of edge 1 whose centre is 0.3 in front of the camera: four
    corners lie behind it, so (reading 8) it has no footprint statistics
    (layered = false, E = 0) and the median gate |0.3 - 0.8| <= h decides:
    the view votes.  Statistics from the in-front corners alone would cover
    the whole image, find the centre pixel's n_samp 101 layered with
    E ~ 100, and the front gate 0.2 > h / 6 would reject."""
    cam = ident_cam(W=64, H=64, f=100.0, cx=32.0, cy=32.0)
    ctr = np.array([0.0, 0.0, 0.3])
    grid, act = grid_for_voxel(ctr, 1.0)
    ns = np.ones((64, 64), np.uint16)
    ns[32, 32] = 101
    v = flat_view(cam, 0.9, 0.1, 0.8, 0.9, nsamp=ns)
    p = oracle.default_params(1.0)
    r = oracle.fuse(act, grid, [v], p, use_nsamp=True)
    assert r["vraw"][0] == 1
    lay, E = oracle.footprint_stats(ns, 0, 63, 0, 63, 101)
    assert lay and 1.0 / (1.0 + 0.05 * E) < 0.2                # what the whole-image statistics would give
