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
    seg = act[H.gpu_segmented(P, v, len(act), lp.tau_cons)].astype(np.uint32)
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


def _thin_kinds(voxel):
    return [("2dgs thin", H.lib_params(voxel, thin=1, rho_thin=5.0, retain_state=1)),
            ("2dgs thin gate 0.6 (no cull)", H.lib_params(voxel, thin=1, rho_thin=5.0, mask_gate=0.6, retain_state=1)),
            ("nerf thin", dv.nerf_params(voxel, "360", thin=1, rho_thin=5.0, retain_state=1)),
            ("thick", H.lib_params(voxel, retain_state=1))]


def _oracle_of(coarse, lp, views, act_ref, rho):
    op = H.oracle_params(lp)
    nerf = lp.variant == 1
    return oracle.fuse(act_ref, coarse.grid, views, op, n_threads=0, variant="nerf" if nerf else "2dgs",
                       thin_rho=rho if lp.thin else None)


def test_thin_sessions_in_batches(coarse):
    """Thin-path sessions (2DGS with and without the chunk cull, NeRF) in one
    batch beside a thick one, with and without the graph, full fusions and then
    appended views folded in by batched updates: every item equals its session
    alone bit for bit and the oracle."""
    import torch
    ctx = dv.Context(0)
    vs = H.upload_views(coarse.views)
    act_ref, rho = oracle.occupancy(coarse.points, coarse.grid, with_rho=True)
    kinds = _thin_kinds(coarse.voxel)
    for use_graph in (False, True):
        _say(f"[case] thin batch graph={use_graph}")
        sess = [(name, lp, H.make_session(coarse, lp, ctx=ctx, max_views=8)[1]) for name, lp in kinds]
        b = dv.Batch(ctx, max_items=len(sess), max_new_views=32, use_graph=use_graph)
        # two views fused, then the other two appended one per batch
        res = [s.alloc_result() for _, _, s in sess]
        b.run([(s, dv.BATCH_FUSE, vs.subset(0, 2), None, 0, r) for (_, _, s), r in zip(sess, res)])
        for k in (2, 3):
            res = [s.alloc_result() for _, _, s in sess]
            b.run([(s, dv.BATCH_UPDATE, vs, k, k, r) for (_, _, s), r in zip(sess, res)])
        torch.cuda.synchronize()
        for (name, lp, s), r in zip(sess, res):
            P, v, c = H.fetch(r)
            _, s2 = H.make_session(coarse, lp, ctx=ctx, max_views=8)
            P2, v2, c2 = H.fetch(s2.fuse_views(vs))
            s2.close()
            assert P.tobytes() == P2.tobytes() and v.tobytes() == v2.tobytes(), name
            assert np.array_equal(c, c2), name
            ref = _oracle_of(coarse, lp, coarse.views, act_ref, rho)
            rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=f"batched {name}")
            _say(f"[ok] thin batch graph={use_graph} {name}: {rep}")
            s.close()
        b.close()


def test_thin_sessions_served(coarse):
    """Thin-path sessions through the continuous-batching server: a full
    fusion, then click updates appending the views; each served result equals
    the session replayed alone and the final one matches the oracle."""
    import torch
    ctx = dv.Context(0)
    vs = H.upload_views(coarse.views)
    act_ref, rho = oracle.occupancy(coarse.points, coarse.grid, with_rho=True)
    srv = dv.Server(ctx, n_streams=2, max_batch=4, use_graph=True)
    grid = dict(origin=coarse.origin, voxel=coarse.voxel, dim=coarse.dim)
    xyz = H.to_dev(coarse.points)
    kinds = _thin_kinds(coarse.voxel)
    served = []
    for name, lp in kinds:
        sid = srv.open_session(grid, xyz, lp, max_views=8, max_view_pixels=coarse.views[0].mask.size)
        outs = []
        n = len(coarse.points)
        r = dict(P=torch.full((n,), -1.0, dtype=torch.float32, device="cuda"),
                 vmask=torch.zeros(n, dtype=torch.int64, device="cuda"),
                 counts=torch.zeros(3, dtype=torch.int64, device="cuda"), seg_bits=None)
        srv.submit(sid, dv.BATCH_FUSE, vs.subset(0, 2), None, 0, r)
        outs.append(r)
        for k in (2, 3):
            r = dict(P=torch.full((n,), -1.0, dtype=torch.float32, device="cuda"),
                     vmask=torch.zeros(n, dtype=torch.int64, device="cuda"),
                     counts=torch.zeros(3, dtype=torch.int64, device="cuda"), seg_bits=None)
            srv.submit(sid, dv.BATCH_UPDATE, vs, k, -1, r)
            outs.append(r)
        served.append((name, lp, outs))
    srv.drain(timeout=120)
    st = srv.stats()
    assert st["failures"] == 0
    torch.cuda.synchronize()
    for name, lp, outs in served:
        _, s = H.make_session(coarse, lp, ctx=ctx, max_views=8)
        alone = [H.fetch(s.fuse_views(vs.subset(0, 2)))]
        for k in (2, 3):
            alone.append(H.fetch(s.update_view(k, vs, k)))
        s.close()
        n_act = len(act_ref)
        for (Pa, va, ca), r in zip(alone, outs):
            Ps, vsv, cs = H.fetch(r)
            assert Ps[:n_act].tobytes() == Pa[:n_act].tobytes() and vsv[:n_act].tobytes() == va[:n_act].tobytes(), name
            assert np.array_equal(cs, ca), name
        ref = _oracle_of(coarse, lp, coarse.views, act_ref, rho)
        Pf, vf, cf = H.fetch(outs[-1])
        rep = H.compare_fusion(Pf[:n_act], vf[:n_act], cf, ref, lp.tau_cons, where=f"served {name}")
        _say(f"[ok] thin served {name}: {rep}")
    srv.close()
