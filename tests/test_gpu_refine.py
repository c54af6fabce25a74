"""GPU parity of the depth refinement of view masks (Eq. depthband,
Eq. gs-bandpass, Eq. nerf-depthweight) through the C ABI against the oracle:
refined planes and statistics bit-exact."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2601_04860_amd as dv  # noqa: E402
import scenes  # noqa: E402
from oracle import mask_refine as R  # noqa: E402
from tests import _helpers as H  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dv.Context(0)


def _prompts(mask, k=3):
    """The k pixels of highest mask value (ties in raster order), as (x, y)."""
    order = np.argsort(-mask.reshape(-1), kind="stable")[:k]
    h, w = mask.shape
    return [(int(i % w), int(i // w)) for i in order]


def _band(ctx, name, mask, d, prompts, in_place=False):
    _say(f"[case] band-pass {name}: {mask.shape} prompts={len(prompts)} in_place={in_place}")
    ref, rst = R.refine_bandpass(mask, d, prompts)
    m_dev = H.to_dev(mask)
    out, st = dv.refine_mask_bandpass(ctx, m_dev, H.to_dev(d), prompts, out=m_dev if in_place else None)
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), f"{name}: {int((got != ref).sum())} pixels differ"
    for k in ("band_min", "band_max", "d_far", "n_surface"):
        assert st[k] == rst[k], (k, st[k], rst[k])
    _say(f"[ok] band-pass {name}: band [{st['band_min']:.4g}, {st['band_max']:.4g}] d_far {st['d_far']:.4g}")


def _minmax(ctx, name, mask, d):
    _say(f"[case] min-max {name}: {mask.shape}")
    ref, rst = R.refine_minmax(mask, d)
    out, st = dv.refine_mask_minmax(ctx, H.to_dev(mask), H.to_dev(d))
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), f"{name}: {int((got != ref).sum())} pixels differ"
    for k in ("z_min", "z_max", "n_surface"):
        assert st[k] == rst[k], (k, st[k], rst[k])
    _say(f"[ok] min-max {name}: z [{st['z_min']:.4g}, {st['z_max']:.4g}]")


def test_refinement_of_the_scene_views(ctx):
    for cfg in ("c1", "c2", "c3"):
        s = scenes.config_scene(cfg)
        for i in (0, len(s.views) - 1):
            v = s.views[i]
            _band(ctx, f"{cfg} view {i}", v.mask, v.dmed, _prompts(v.mask))
            _minmax(ctx, f"{cfg} view {i}", v.mask, v.dmed)
    v = scenes.config_scene("c1").views[1]
    _band(ctx, "c1 view 1 in place", v.mask, v.dmed, _prompts(v.mask, 5), in_place=True)


def test_refinement_special_cases(ctx):
    rng = np.random.default_rng(21)
    for (h, w) in ((1, 1), (3, 517), (64, 65), (257, 129)):
        d = (0.5 + rng.random((h, w)) * 4).astype(np.float32)
        d[rng.random((h, w)) < 0.1] = 0.0
        d[0, 0] = 1.5
        m = rng.random((h, w)).astype(np.float32)
        _band(ctx, f"ragged {h}x{w}", m, d, [(0, 0)])
        _minmax(ctx, f"ragged {h}x{w}", m, d)
    # the band reaches d_far: denominator floor
    d = np.full((4, 4), 2.0, np.float32)
    d[0, 0] = 1.0
    _band(ctx, "floor", np.ones((4, 4), np.float32), d, [(1, 1)])
    # flat depth: every surface pixel keeps its mask
    d = np.full((5, 7), 3.0, np.float32)
    d[2, 3] = 0.0
    _minmax(ctx, "flat", rng.random((5, 7)).astype(np.float32), d)
    # the two ranks of d_far on both sides of a gap in depth (each counted in
    # its own histogram), with a fraction between them
    m = 40 * 50
    i = int(np.floor(0.98 * (m - 1)))
    d = np.concatenate([1 + rng.random(i + 1), 50 + rng.random(m - i - 1)]).astype(np.float32)
    d = rng.permutation(d).reshape(40, 50)
    _band(ctx, "d_far across a gap", rng.random((40, 50)).astype(np.float32), d, [(0, 0)])
    # NaN and infinite depths are pixels without a surface
    d = (1 + rng.random((33, 31)) * 2).astype(np.float32)
    d[::5, ::3] = np.nan
    d[1::7, 2::4] = np.inf
    d[16, 15] = 1.25
    _band(ctx, "non-finite", rng.random((33, 31)).astype(np.float32), d, [(3, 4)])


def test_refinement_rejects_bad_inputs(ctx):
    m = H.to_dev(np.ones((8, 8), np.float32))
    with pytest.raises(dv.DivasError):   # no surface
        dv.refine_mask_minmax(ctx, m, H.to_dev(np.zeros((8, 8), np.float32)))
    d = np.full((8, 8), 2.0, np.float32)
    d[4, 4] = 0.0
    d[1, 1] = 0.0
    with pytest.raises(dv.DivasError):   # neither the prompt nor the centre has a surface
        dv.refine_mask_bandpass(ctx, m, H.to_dev(d), [(1, 1)])
    with pytest.raises(dv.DivasError):   # prompt outside the view
        dv.refine_mask_bandpass(ctx, m, H.to_dev(np.ones((8, 8), np.float32)), [(8, 0)])


def test_fusion_with_refined_masks(ctx):
    """The refined planes feed the fusion: the c1 scene fused with band-pass
    masks matches the oracle fused with the oracle's refined masks."""
    s = scenes.config_scene("c1")
    lp = H.lib_params(s.voxel)
    op = H.oracle_params(lp)
    views = []
    vs = dv.ViewSet()
    for v in s.views:
        pr = _prompts(v.mask)
        ref, _ = R.refine_bandpass(v.mask, v.dmed, pr)
        out, _ = dv.refine_mask_bandpass(ctx, H.to_dev(v.mask), H.to_dev(v.dmed), pr)
        assert np.array_equal(out.cpu().numpy(), ref)
        vs.add(v.cam, v.d_cam, out, H.to_dev(v.dmin), H.to_dev(v.dmed), H.to_dev(v.dmax))
        views.append(v._replace(mask=ref) if hasattr(v, "_replace") else _with_mask(v, ref))
    _, sess = H.make_session(s, lp, ctx=ctx)
    act = sess.active_indices()
    P, vm, c = H.fetch(sess.fuse_views(vs))
    refd = oracle.fuse(act.astype(np.uint32), s.grid, views, op, n_threads=0)
    rep = H.compare_fusion(P, vm, c, refd, lp.tau_cons, where="c1 refined")
    _say(f"[ok] fusion with refined masks: {rep}")
    sess.close()


def _with_mask(v, mask):
    import copy
    w = copy.copy(v)
    w.mask = mask
    return w
