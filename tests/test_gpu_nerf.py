"""GPU parity of the NeRF path (Alg. nerf-fusion, and Alg. nerf-thin) through
the C ABI against the oracle, under both depth readings: the tuple as camera Z
(the default) and as distances along the pixel rays.  Same bar as the 2DGS
path: view bitmasks, segmentation and labels bit-exact, float32 P within 1e-5
relative of the binary64 oracle."""
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


def ray_views(views):
    """The views with their ray-distance depth planes (NeRF depth semantics)."""
    return [v.as_ray_depth() for v in views]


def _case(scene, name, column, use_nsamp=False, ray=False, thin=False, **kw):
    views = ray_views(scene.views) if ray else scene.views
    lp = dv.nerf_params(scene.voxel, column, nerf_ray_depths=int(ray), thin=int(thin), **kw)
    op = H.oracle_params(lp)
    _say(f"[case] nerf {name}: column={column} nsamp={use_nsamp} ray={ray} thin={thin} {kw}")
    ctx, sess = H.make_session(scene, lp, max_views=len(views))
    act = sess.active_indices()
    P, v, c = H.fetch(sess.fuse_views(H.upload_views(views, use_nsamp=use_nsamp)))
    rho = None
    if thin:
        act_ref, rho = oracle.occupancy(scene.points, scene.grid, with_rho=True)
        assert np.array_equal(act, act_ref.astype(np.int64))
    ref = oracle.fuse(act.astype(np.uint32), scene.grid, views, op, use_nsamp=use_nsamp, n_threads=0, variant="nerf",
                      thin_rho=rho)
    rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=name)
    assert int(ref["counts"][2]) > 0, "no vote at all: the case tests nothing"
    if thin:
        plain = oracle.fuse(act.astype(np.uint32), scene.grid, views, op, use_nsamp=use_nsamp, n_threads=0,
                            variant="nerf")
        rep["thin_gained"] = int((ref["vraw"] != plain["vraw"]).sum())
    lpts = np.asarray(scene.points, np.float32)
    lab = sess.label_points(H.to_dev(lpts)).cpu().numpy()
    seg = act[H.gpu_segmented(P, v, len(act), lp.tau_cons)].astype(np.uint32)
    assert np.array_equal(lab, oracle.label(lpts, scene.grid, seg))
    _say(f"[ok] nerf {name}: votes={int(ref['counts'][2])} {rep}")
    sess.close()
    return rep


@pytest.fixture(scope="module")
def c1():
    return scenes.config_scene("c1")


def test_nerf_c1_columns_and_samples(c1):
    _case(c1, "c1 360", "360")
    _case(c1, "c1 llff", "llff")
    _case(c1, "c1 360 n_samp", "360", use_nsamp=True)
    _case(c1, "c1 gate 0", "360", mask_gate=0.0, lambda_range=0.5)


def test_nerf_c1_ray_depths(c1):
    _case(c1, "c1 360 ray", "360", ray=True)
    _case(c1, "c1 llff ray n_samp", "llff", ray=True, use_nsamp=True)


def test_nerf_c2_full():
    c2 = scenes.config_scene("c2")
    _case(c2, "c2 llff", "llff")
    _case(c2, "c2 llff ray", "llff", ray=True)


@pytest.fixture(scope="module")
def coarse():
    return scenes.make_tiny_sphere(dim=32, n_points=20000, n_views=4, width=256, height=192, focal=300.0, seed=1)


def test_nerf_thin_path_matches_the_oracle(coarse):
    """Alg. nerf-thin on a coarse grid whose voxels cover 40-60 pixels per
    view (density floor lowered to the scene's point counts)."""
    rep = _case(coarse, "coarse 360 thin", "360", thin=True, rho_thin=5.0)
    assert rep["thin_gained"] > 20
    _case(coarse, "coarse llff thin n_samp", "llff", thin=True, rho_thin=5.0, use_nsamp=True)
    _case(coarse, "coarse 360 thin ray", "360", thin=True, rho_thin=5.0, ray=True)
    _case(coarse, "coarse 360 thin gate 0", "360", thin=True, rho_thin=5.0, mask_gate=0.0)
    _case(coarse, "coarse 360 thin no cover", "360", thin=True, rho_thin=5.0, rho_cover=0.0)


def test_nerf_incremental_and_batched_equal_full(c1):
    views = c1.views
    vs = H.upload_views(views)
    n = len(views)
    lp = dv.nerf_params(c1.voxel, "360", mask_gate=0.0, retain_state=1)
    ctx, s = H.make_session(c1, lp, max_views=8)
    s.fuse_views(H.upload_views(views[:1]))
    for k in range(1, n):
        res = s.update_view(k, vs, k)
    P_inc, v_inc, c_inc = H.fetch(res)
    ctx2, s2 = H.make_session(c1, dv.nerf_params(c1.voxel, "360", mask_gate=0.0), ctx=ctx)
    P_full, v_full, c_full = H.fetch(s2.fuse_views(vs))
    assert P_inc.tobytes() == P_full.tobytes() and v_inc.tobytes() == v_full.tobytes()
    assert np.array_equal(c_inc, c_full)
    # a batch holding a NeRF session and a 2DGS session equals each alone
    lp_g = dv.default_params(c1.voxel)
    _, s3 = H.make_session(c1, lp_g, ctx=ctx)
    vs_g = H.upload_views(c1.views)
    b = dv.Batch(ctx, max_items=2, max_new_views=16)
    r2, r3 = s2.alloc_result(), s3.alloc_result()
    b.run([(s2, dv.BATCH_FUSE, vs, None, 0, r2), (s3, dv.BATCH_FUSE, vs_g, None, 0, r3)])
    P2, v2, c2 = H.fetch(r2)
    assert P2.tobytes() == P_full.tobytes() and v2.tobytes() == v_full.tobytes() and np.array_equal(c2, c_full)
    _, s4 = H.make_session(c1, lp_g, ctx=ctx)
    P4, v4, c4 = H.fetch(s4.fuse_views(vs_g))
    P3, v3, c3 = H.fetch(r3)
    assert P3.tobytes() == P4.tobytes() and v3.tobytes() == v4.tobytes() and np.array_equal(c3, c4)
    b.close()
    for x in (s, s2, s3, s4):
        x.close()


def test_nerf_rejects_bad_params(c1):
    with pytest.raises(dv.DivasError):
        H.make_session(c1, dv.nerf_params(c1.voxel, "360", differentiable=1))
    with pytest.raises(dv.DivasError):
        H.make_session(c1, dv.nerf_params(c1.voxel, "360", variant=2))
    with pytest.raises(dv.DivasError):
        H.make_session(c1, dv.nerf_params(c1.voxel, "360", lambda_range=-1.0))
