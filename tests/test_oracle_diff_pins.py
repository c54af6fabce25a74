"""Pins of the differentiable oracle variant: its analytic gradient against
central finite differences of its own forward (steps exact in float32), against
an independent float64 autograd implementation, and the hard-gate limit."""
import math

import numpy as np
import pytest

import oracle
import scenes
from oracle import grad_ref
from scenes import View


def _scene():
    s = scenes.make_diff_scene(dim=32, n_points=5000, width=64, height=48, focal=50.0)
    act = oracle.occupancy(s.points, s.grid)
    g = s.dim
    ijk = np.stack([act % g, (act // g) % g, act // (g * g)], 1)
    crop = np.all(ijk >= 16, 1)  # positive octant: holds sphere surface
    return s, act[crop]


def _params(s, **kw):
    kw.setdefault("soft_width", 0.01)
    return oracle.default_params(s.voxel, mask_gate=0.0, **kw)


def _with(views, s_idx, key, arr):
    out = []
    for i, v in enumerate(views):
        if i != s_idx:
            out.append(v)
            continue
        d = dict(cam=v.cam, d_cam=v.d_cam, mask=v.mask, dmin=v.dmin, dmed=v.dmed, dmax=v.dmax, logit=v.logit)
        d[key] = arr
        out.append(View(**d))
    return out


def test_gradient_matches_independent_autograd():
    s, act = _scene()
    p = _params(s)
    rng = np.random.default_rng(7)
    gP = rng.normal(size=len(act))
    P_c, _, _ = oracle.fuse_diff(act, s.grid, s.views, p)
    P_t, gt = grad_ref.grads(act, s.grid, s.views, p, gP)
    assert np.allclose(P_c, P_t, rtol=1e-12, atol=1e-14)
    assert (P_c > 0).sum() > 100
    gc = oracle.fuse_diff_grad(act, s.grid, s.views, p, gP)
    for k in ("logit", "dmin", "dmed", "dmax"):
        for a, b in zip(gc[k], gt[k]):
            scale = np.abs(b).max() + 1e-30
            assert np.allclose(a, b, rtol=1e-7, atol=1e-7 * scale), k
        assert sum(np.count_nonzero(a) for a in gc[k]) > 20, k


@pytest.mark.parametrize("key,step", [("logit", 2.0 ** -8), ("dmin", 2.0 ** -14),
                                      ("dmed", 2.0 ** -14), ("dmax", 2.0 ** -14)])
def test_gradient_matches_central_differences(key, step):
    s, act = _scene()
    p = _params(s)
    rng = np.random.default_rng(11)
    gP = rng.normal(size=len(act))
    P0 = oracle.fuse_diff(act, s.grid, s.views, p)[0]
    # difference P voxel by voxel before the dot product: full precision
    loss = lambda views: float(np.dot(gP, oracle.fuse_diff(act, s.grid, views, p)[0] - P0))
    gc = oracle.fuse_diff_grad(act, s.grid, s.views, p, gP)
    checked = 0
    gmax = max(np.abs(g).max() for g in gc[key])
    for si in range(len(s.views)):
        g = gc[key][si]
        order = np.argsort(-np.abs(g).ravel())[:6]
        cand = [np.unravel_index(i, g.shape) for i in order if abs(g.ravel()[i]) > 1e-3 * gmax]
        for (y, x) in cand:
            base = getattr(s.views[si], key)
            vals = []
            for sgn in (+1, -1):
                arr = base.copy()
                nv = np.float32(float(arr[y, x]) + sgn * step)
                assert float(nv) == float(arr[y, x]) + sgn * step  # exact perturbation
                arr[y, x] = nv
                vals.append(loss(_with(s.views, si, key, arr)))
            f0 = 0.0
            fwd, bwd = (vals[0] - f0) / step, (f0 - vals[1]) / step
            if abs(fwd - bwd) > 0.05 * (abs(fwd) + abs(bwd) + 1e-12):
                continue  # a hard gate or clamp kink inside the step
            fd = (vals[0] - vals[1]) / (2 * step)
            assert math.isclose(fd, g[y, x], rel_tol=2e-5, abs_tol=1e-6 * gmax + 6e-16 / step), (si, y, x)
            checked += 1
    assert checked >= 8


def test_soft_width_limit_is_hard_R2():
    s, act = _scene()
    p = _params(s, soft_width=1e-12)
    P_soft, _, _ = oracle.fuse_diff(act, s.grid, s.views, p)
    hard_views = [View(cam=v.cam, d_cam=v.d_cam, mask=(1 / (1 + np.exp(-v.logit.astype(np.float64)))).astype(np.float32),
                       dmin=v.dmin, dmed=v.dmed, dmax=v.dmax) for v in s.views]
    r = oracle.fuse(act, s.grid, hard_views, oracle.default_params(s.voxel, mask_gate=0.0))
    # identical except where sigmoid(logit) was rounded to float32 for the hard run
    assert np.allclose(P_soft, r["P"], rtol=1e-6, atol=1e-7)
    assert np.array_equal(P_soft > 0, r["P"] > 0)
