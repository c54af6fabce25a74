"""Several target objects of one scene fused together (divas_fuse_targets over
a session and target sessions of it): every target's outputs and state equal
its fusion alone bit for bit and match the oracle; the error paths."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2601_04860_amd as dv  # noqa: E402
import scenes  # noqa: E402
from tests import _helpers as H  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _host_views(views, t):
    return [scenes.View(cam=v.cam, d_cam=v.d_cam, mask=v.masks[t], dmin=v.dmin, dmed=v.dmed, dmax=v.dmax,
                        nsamp=v.nsamp) for v in views]


@pytest.fixture(scope="module")
def multi():
    return scenes.make_grid_scene(11, 64, 5, 160, 120, 4, n_points=40000)


def _setup(sc, ctx, lp, T, use_nsamp=False, max_views=None):
    grid = dict(origin=sc.origin, voxel=sc.voxel, dim=sc.dim)
    xyz = H.to_dev(sc.points)
    mv = max_views or len(sc.views) + 2
    mp = max(v.mask.size for v in sc.views)
    base = dv.Session(ctx, grid, xyz, params=lp, max_views=mv, max_view_pixels=mp)
    sess = [base] + [dv.Session.target(base, params=lp, max_views=mv, max_view_pixels=mp) for _ in range(T - 1)]
    vs0 = H.upload_views(sc.views, use_nsamp=use_nsamp)
    sets = [vs0.with_masks([H.to_dev(v.masks[t]) for v in sc.views]) for t in range(T)]
    return base, sess, sets, xyz


def _check_targets(sc, ctx, lp, T, name, use_nsamp=False, oracle_targets=None, schedule="together"):
    _say(f"[case] targets {name}: T={T} nsamp={use_nsamp} schedule={schedule}")
    base, sess, sets, xyz = _setup(sc, ctx, lp, T, use_nsamp)
    res = [s.alloc_result() for s in sess]
    dv.fuse_targets(sess, sets, res, schedule=schedule)
    act = base.active_indices()
    op = H.oracle_params(lp)
    pts = np.asarray(sc.points, np.float32)
    for t in range(T):
        P, v, c = H.fetch(res[t])
        _, alone = H.make_session(sc, lp, ctx=ctx, max_views=len(sc.views) + 2)
        P2, v2, c2 = H.fetch(alone.fuse_views(sets[t]))
        alone.close()
        assert P.tobytes() == P2.tobytes() and v.tobytes() == v2.tobytes(), f"{name}: target {t}"
        assert np.array_equal(c, c2), f"{name}: target {t} counts"
        if oracle_targets is None or t in oracle_targets:
            ref = oracle.fuse(act.astype(np.uint32), sc.grid, _host_views(sc.views, t), op, use_nsamp=use_nsamp,
                              n_threads=0, variant="nerf" if lp.variant == 1 else "2dgs")
            rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=f"{name} target {t}")
            seg = act[H.gpu_segmented(P, v, len(act), lp.tau_cons)].astype(np.uint32)
            lab = sess[t].label_points(xyz).cpu().numpy()
            assert np.array_equal(lab, oracle.label(pts, sc.grid, seg)), f"{name}: target {t} labels"
            _say(f"[ok] targets {name} target {t}: {rep}")
    for s in reversed(sess):
        s.close()


def test_targets_equal_alone_and_oracle(multi):
    """The shared kernel under both gate readings (forced together under the
    default gate, where the automatic schedule fuses one after another), and
    the automatic schedule."""
    ctx = dv.Context(0)
    lp = dv.default_params(multi.voxel)
    _check_targets(multi, ctx, lp, 4, "R1")
    _check_targets(multi, ctx, dv.default_params(multi.voxel, mask_gate=0.0), 3, "R2")
    _check_targets(multi, ctx, lp, 2, "R1 n_samp", use_nsamp=True)
    _check_targets(multi, ctx, dv.default_params(multi.voxel, mask_gate=0.0), 4, "R2 n_samp", use_nsamp=True)
    _check_targets(multi, ctx, lp, 3, "R1 auto", schedule="auto")
    _check_targets(multi, ctx, dv.default_params(multi.voxel, mask_gate=0.0), 2, "R2 auto", schedule="auto")
    _check_targets(multi, ctx, lp, 2, "R1 one by one", schedule="one_by_one")


def test_targets_fallback_and_updates(multi):
    """NeRF parameters fuse the targets one after another (same results);
    target sessions take click updates, folded bit for bit."""
    ctx = dv.Context(0)
    _check_targets(multi, ctx, dv.nerf_params(multi.voxel, "360"), 3, "NeRF (one after another)")
    lp = dv.default_params(multi.voxel, retain_state=1)
    base, sess, sets, xyz = _setup(multi, ctx, lp, 3)
    n = len(multi.views)
    res = [s.alloc_result() for s in sess]
    dv.fuse_targets(sess, [v.subset(0, n - 1) for v in sets], res)
    for t, s in enumerate(sess):  # append the last view to each target
        r = s.update_view(n - 1, sets[t], n - 1)
        P, v, c = H.fetch(r)
        _, alone = H.make_session(multi, dv.default_params(multi.voxel), ctx=ctx, max_views=n + 2)
        P2, v2, c2 = H.fetch(alone.fuse_views(sets[t]))
        alone.close()
        assert P.tobytes() == P2.tobytes() and v.tobytes() == v2.tobytes() and np.array_equal(c, c2)
    for s in reversed(sess):
        s.close()


def test_targets_rejections(multi):
    ctx = dv.Context(0)
    lp = dv.default_params(multi.voxel)
    base, sess, sets, xyz = _setup(multi, ctx, lp, 2)
    other, _ = None, None
    _, other = H.make_session(multi, lp, ctx=ctx)
    res = [s.alloc_result() for s in sess]
    with pytest.raises(dv.DivasError):   # a session of another scene
        dv.fuse_targets([sess[0], other], sets, res)
    bad = sets[1].with_masks([H.to_dev(v.masks[1]) for v in multi.views])
    bad.maps[0] = dv.ViewMaps(bad.maps[0].mask, bad.maps[0].d_ref, bad.maps[0].d_ref, bad.maps[0].d_max, None)
    with pytest.raises(dv.DivasError):   # depth planes that differ between targets
        dv.fuse_targets(sess, [sets[0], bad], res)
    with pytest.raises(dv.DivasError):   # a repeated session
        dv.fuse_targets([sess[0], sess[0]], sets, res)
    with pytest.raises(ValueError):      # an unknown schedule
        dv.fuse_targets(sess, sets, res, schedule="sideways")
    with pytest.raises(dv.DivasError):   # the base cannot be rebuilt while targets live
        base.rebuild(xyz)
    with pytest.raises(dv.DivasError):   # nor destroyed
        dv._check(dv.lib().divas_session_destroy(base.handle), "destroy")
    with pytest.raises(dv.DivasError):   # a target is never rebuilt
        sess[1].rebuild(xyz)
    with pytest.raises(dv.DivasError):   # a target of a target
        dv.Session.target(sess[1], params=lp)
    sess[1].close()
    base.rebuild(xyz)                    # allowed once its targets are gone
    base.close()
    other.close()


def test_targets_serving_scene_full_size():
    """The largest scene of the serving workload (512^3, 16 views 1264x832,
    8 targets): every target equal to its fusion alone, two against the
    oracle."""
    wl = scenes.config_scene("c5")
    sc = wl["scenes"][3]
    ctx = dv.Context(0)
    _check_targets(sc, ctx, dv.default_params(sc.voxel), 8, "serving 512^3", oracle_targets=(0, 7))
    _check_targets(sc, ctx, dv.default_params(sc.voxel, mask_gate=0.0), 8, "serving 512^3 gate 0",
                   oracle_targets=(3,), schedule="auto")
