"""GPU parity of the thin-structure fallback (Alg. gs-thin, Eq. behind-gate)
against the oracle, on a coarse grid whose voxels cover 40-60 pixels in each
view.  Same bar as the thick path: view bitmasks, segmentation and labels
bit-exact, float32 P within 1e-5 relative of the binary64 oracle."""
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


@pytest.fixture(scope="module")
def coarse():
    return scenes.make_tiny_sphere(dim=32, n_points=20000, n_views=4, width=256, height=192, focal=300.0, seed=1)


def _case(s, name, use_nsamp=False, points=None, **kw):
    pts = s.points if points is None else points
    lp = H.lib_params(s.voxel, thin=1, **kw)
    op = H.oracle_params(lp)
    _say(f"[case] thin {name}: nsamp={use_nsamp} {kw}")
    ctx, sess = H.make_session(s, lp, points=pts)
    act = sess.active_indices()
    act_ref, rho = oracle.occupancy(pts, s.grid, with_rho=True)
    assert np.array_equal(act, act_ref.astype(np.int64))
    P, v, c = H.fetch(sess.fuse_views(H.upload_views(s.views, use_nsamp=use_nsamp)))
    ref = oracle.fuse(act_ref, s.grid, s.views, op, use_nsamp=use_nsamp, n_threads=0, thin_rho=rho)
    plain = oracle.fuse(act_ref, s.grid, s.views, op, use_nsamp=use_nsamp, n_threads=0)
    gained = int((ref["vraw"] != plain["vraw"]).sum())
    rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=name)
    pts32 = np.asarray(pts, np.float32)
    lab = sess.label_points(H.to_dev(pts32)).cpu().numpy()
    seg = act[P[:len(act)].astype(np.float64) >= lp.tau_cons].astype(np.uint32)
    assert np.array_equal(lab, oracle.label(pts32, s.grid, seg))
    _say(f"[ok] thin {name}: voxels with thin votes={gained} {rep}")
    sess.close()
    return gained


def test_thin_fallback_matches_the_oracle(coarse):
    assert _case(coarse, "default floor", ) > 50
    assert _case(coarse, "rho 5", rho_thin=5.0) > 50
    _case(coarse, "rho 10", rho_thin=10.0)
    assert _case(coarse, "rho 5 n_samp", use_nsamp=True, rho_thin=5.0) > 0
    _case(coarse, "gate 0", rho_thin=5.0, mask_gate=0.0)


def test_thin_density_follows_a_rebuild(coarse):
    rng = np.random.default_rng(3)
    pts = coarse.points[rng.permutation(len(coarse.points))[:12000]]
    _case(coarse, "rebuilt subset", points=pts, rho_thin=4.0)


def test_thin_rejections(coarse):
    ctx = dv.Context(0)
    with pytest.raises(dv.DivasError):   # density needs point counts
        H.make_session(coarse, H.lib_params(coarse.voxel, thin=1), ctx=ctx,
                       opacity=np.ones(len(coarse.points), np.float32))
    with pytest.raises(dv.DivasError):   # a zero score must not vote
        H.make_session(coarse, H.lib_params(coarse.voxel, thin=1, tau_thin=0.0), ctx=ctx)
    with pytest.raises(dv.DivasError):
        H.make_session(coarse, dv.nerf_params(coarse.voxel, "360", thin=1, tau_thin=0.0), ctx=ctx)
    with pytest.raises(dv.DivasError):
        H.make_session(coarse, H.lib_params(coarse.voxel, thin=1, rho_occ=-1.0), ctx=ctx)
    _, s = H.make_session(coarse, H.lib_params(coarse.voxel, thin=1), ctx=ctx)
    b = dv.Batch(ctx, max_items=1, max_new_views=8)
    with pytest.raises(dv.DivasError):
        b.run([(s, dv.BATCH_FUSE, H.upload_views(coarse.views), None, 0, s.alloc_result())])
    b.close()
    s.close()


def test_thin_incremental_equals_full(coarse):
    """Folding views one by one into the resident accumulators equals the
    full fusion bit for bit with the thin fallback too."""
    vs = H.upload_views(coarse.views)
    lp = H.lib_params(coarse.voxel, thin=1, rho_thin=5.0, retain_state=1)
    ctx, s = H.make_session(coarse, lp, max_views=8)
    s.fuse_views(H.upload_views(coarse.views[:1]))
    for k in range(1, len(coarse.views)):
        res = s.update_view(k, vs, k)
    P_inc, v_inc, c_inc = H.fetch(res)
    _, s2 = H.make_session(coarse, H.lib_params(coarse.voxel, thin=1, rho_thin=5.0), ctx=ctx)
    P_full, v_full, c_full = H.fetch(s2.fuse_views(vs))
    assert P_inc.tobytes() == P_full.tobytes() and v_inc.tobytes() == v_full.tobytes()
    assert np.array_equal(c_inc, c_full)
    s.close()
    s2.close()
