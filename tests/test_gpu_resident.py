"""Resident outputs (params.resident_outputs): a fold into the buffers of the
session's previous fusion call writes only the chunks the new view can reach,
and keeps the counts as running totals.  Every result equals the one written
in full (fresh buffers, resident outputs off) bit for bit, alone, in batches
and through the server; the final fusion matches the oracle; any other call
writes every entry."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2601_04860_amd as dv  # noqa: E402
import scenes  # noqa: E402
from tests import _helpers as H  # noqa: E402

SENTINEL = -7.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c2():
    return scenes.config_scene("c2")


def _params(sc, resident, **kw):
    return dv.default_params(sc.voxel, retain_state=1, resident_outputs=1 if resident else 0, **kw)


def _reference(sc, ctx, lp_kw, n0):
    """Fresh buffers for every call, resident outputs off: P, vmask, counts
    after the full fusion of views [0, n0) and after each appended view."""
    _, s = H.make_session(sc, _params(sc, False, **lp_kw), ctx=ctx)
    vs = H.upload_views(sc.views)
    outs = [H.fetch(s.fuse_views(vs.subset(0, n0)))]
    for k in range(n0, len(sc.views)):
        outs.append(H.fetch(s.update_view(k, vs, k)))
    s.close()
    return outs


def _same(a, b, where):
    P, v, c = a
    P2, v2, c2 = b
    assert P.tobytes() == P2.tobytes(), f"{where}: P"
    assert v.tobytes() == v2.tobytes(), f"{where}: vmask"
    assert np.array_equal(c, c2), f"{where}: counts {c} vs {c2}"


@pytest.mark.parametrize("gate", [0.5, 0.0])
def test_resident_folds_equal_full_writes(c2, gate):
    """Append the views one by one into the same buffers: every step equals
    the full write; the labels follow; the last fusion matches the oracle.  A
    sentinel planted in P before one fold shows that entries of chunks the new
    view cannot reach are left alone (and only those)."""
    ctx = dv.Context(0)
    n0 = 3
    _say(f"[case] resident folds gate={gate}")
    ref = _reference(c2, ctx, dict(mask_gate=gate), n0)
    lp = _params(c2, True, mask_gate=gate)
    _, s = H.make_session(c2, lp, ctx=ctx)
    vs = H.upload_views(c2.views)
    res = s.fuse_views(vs.subset(0, n0))
    _same(H.fetch(res), ref[0], "full fusion")
    n_act = s.info()["n_active"]
    for j, k in enumerate(range(n0, len(c2.views))):
        planted = j == 1
        if planted:
            res["P"][:n_act] = SENTINEL
        s.update_view(k, vs, k, res)
        P, v, c = H.fetch(res)
        if planted:
            written = P[:n_act] != SENTINEL
            hot = s.fusion_work()["hot_chunks"]
            assert 0 < written.sum() <= min(hot * 64, n_act), (int(written.sum()), hot, n_act)
            if gate > 0:  # the default gate leaves most chunks out of the new view's reach
                assert written.sum() < n_act // 2, (int(written.sum()), n_act)
            assert np.array_equal(P[:n_act][written], ref[j + 1][0][:n_act][written]), "written entries"
            assert np.array_equal(c, ref[j + 1][2]), "running totals"
            assert v.tobytes() == ref[j + 1][1].tobytes(), "vmask"
            _say(f"[ok] fold {k}: {int(written.sum())} of {n_act} entries written ({hot} chunks)")
            # put the untouched values back, as a caller that keeps its buffers has them
            res["P"][:n_act] = H.to_dev(ref[j + 1][0][:n_act])
        else:
            _same((P, v, c), ref[j + 1], f"fold {k}")
    act = s.active_indices()
    pts = np.asarray(c2.points, np.float32)
    P, v, c = H.fetch(res)
    seg = act[H.gpu_segmented(P, v, len(act), lp.tau_cons)].astype(np.uint32)
    assert np.array_equal(s.label_points(H.to_dev(pts)).cpu().numpy(), oracle.label(pts, c2.grid, seg))
    ref_o = oracle.fuse(act.astype(np.uint32), c2.grid, c2.views, H.oracle_params(lp), n_threads=0)
    rep = H.compare_fusion(P, v, c, ref_o, lp.tau_cons, where=f"resident gate {gate}")
    _say(f"[ok] resident folds gate={gate}: {rep}")
    s.close()


def test_resident_outputs_fall_back_to_full_writes(c2):
    """Other buffers, a full fusion in between, a rebuild: every entry is
    written (no sentinel survives), and the results equal the full write."""
    ctx = dv.Context(0)
    n0 = 3
    ref = _reference(c2, ctx, {}, n0)
    _, s = H.make_session(c2, _params(c2, True), ctx=ctx)
    vs = H.upload_views(c2.views)
    n_act = s.info()["n_active"]
    res = s.fuse_views(vs.subset(0, n0))
    other = s.alloc_result()
    other["P"][:n_act] = SENTINEL
    s.update_view(n0, vs, n0, other)  # not the previous call's buffers
    assert not (H.fetch(other)[0][:n_act] == SENTINEL).any()
    _same(H.fetch(other), ref[1], "other buffers")
    # back to res: not the previous call's buffers either
    res["P"][:n_act] = SENTINEL
    s.update_view(n0 + 1, vs, n0 + 1, res)
    assert not (H.fetch(res)[0][:n_act] == SENTINEL).any()
    _same(H.fetch(res), ref[2], "buffers of an older call")
    # a rebuild in between: full writes again
    s.rebuild(s._keep_xyz[0])
    s.fuse_views(vs.subset(0, n0), res)
    _same(H.fetch(res), ref[0], "after a rebuild")
    s.update_view(n0, vs, n0, res)  # resident again: same buffers, nothing in between
    _same(H.fetch(res), ref[1], "resident after the rebuild")
    s.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_resident_outputs_in_batches(c2, use_graph):
    """Batched updates of sessions with and without resident outputs, each
    into its previous buffers: every item equals its full-write sequence."""
    ctx = dv.Context(0)
    n0 = 3
    kinds = [("resident", True, 0.5), ("resident gate 0", True, 0.0), ("full writes", False, 0.5)]
    refs = {name: _reference(c2, ctx, dict(mask_gate=g), n0) for name, _, g in kinds}
    vs = H.upload_views(c2.views)
    sess = [(name, H.make_session(c2, _params(c2, r, mask_gate=g), ctx=ctx)[1]) for name, r, g in kinds]
    res = [s.alloc_result() for _, s in sess]
    b = dv.Batch(ctx, max_items=len(sess), max_new_views=32, use_graph=use_graph)
    b.run([(s, dv.BATCH_FUSE, vs.subset(0, n0), None, 0, r) for (_, s), r in zip(sess, res)])
    for (name, _), r in zip(sess, res):
        _same(H.fetch(r), refs[name][0], f"{name} batched fusion")
    for j, k in enumerate(range(n0, len(c2.views))):
        b.run([(s, dv.BATCH_UPDATE, vs, k, k, r) for (_, s), r in zip(sess, res)])
        for (name, _), r in zip(sess, res):
            _same(H.fetch(r), refs[name][j + 1], f"{name} batched update {k} graph={use_graph}")
    _say(f"[ok] resident batches graph={use_graph}")
    b.close()
    for _, s in sess:
        s.close()


def test_resident_outputs_served(c2):
    """Click updates through the server into one result per session: each
    session's final result equals its full-write sequence."""
    import torch
    ctx = dv.Context(0)
    n0 = 3
    ref = _reference(c2, ctx, {}, n0)
    vs = H.upload_views(c2.views)
    srv = dv.Server(ctx, n_streams=2, max_batch=4, use_graph=True)
    grid = dict(origin=c2.origin, voxel=c2.voxel, dim=c2.dim)
    xyz = H.to_dev(c2.points)
    results = []
    for _ in range(3):
        sid = srv.open_session(grid, xyz, _params(c2, True), max_views=len(c2.views),
                               max_view_pixels=c2.views[0].mask.size)
        n = len(c2.points)
        r = dict(P=torch.full((n,), -1.0, dtype=torch.float32, device="cuda"),
                 vmask=torch.zeros(n, dtype=torch.int64, device="cuda"),
                 counts=torch.zeros(3, dtype=torch.int64, device="cuda"), seg_bits=None)
        srv.submit(sid, dv.BATCH_FUSE, vs.subset(0, n0), None, 0, r)
        for k in range(n0, len(c2.views)):
            srv.submit(sid, dv.BATCH_UPDATE, vs, k, -1, r)
        results.append(r)
    srv.drain(timeout=120)
    assert srv.stats()["failures"] == 0
    torch.cuda.synchronize()
    n_act = len(ref[-1][0])
    for r in results:
        P, v, c = H.fetch(r)
        _same((P[:n_act], v[:n_act], c), ref[-1], "served")
    srv.close()


@pytest.mark.parametrize("kind", ["2dgs thin", "nerf thin", "nerf"])
def test_resident_outputs_thin_and_nerf(kind):
    """Resident outputs with the thin paths (the block-shared sweep kernel)
    and the NeRF thick path, on the coarse tiny-sphere grid: folds into the
    same buffers equal the full writes, and the final fusion matches the
    oracle."""
    sc = scenes.make_tiny_sphere(dim=32, n_points=20000, n_views=4, width=256, height=192, focal=300.0, seed=1)
    ctx = dv.Context(0)

    def params(resident):
        kw = dict(retain_state=1, resident_outputs=1 if resident else 0)
        if kind == "2dgs thin":
            return dv.default_params(sc.voxel, thin=1, rho_thin=5.0, **kw)
        if kind == "nerf thin":
            return dv.nerf_params(sc.voxel, "360", thin=1, rho_thin=5.0, **kw)
        return dv.nerf_params(sc.voxel, "360", **kw)

    vs = H.upload_views(sc.views)
    outs = {}
    for resident in (False, True):
        _, s = H.make_session(sc, params(resident), ctx=ctx)
        res = s.alloc_result()
        seq = [H.fetch(s.fuse_views(vs.subset(0, 1), res if resident else None))]
        for k in range(1, len(sc.views)):
            seq.append(H.fetch(s.update_view(k, vs, k, res if resident else None)))
        if resident:
            act = s.active_indices()
        s.close()
        outs[resident] = seq
    for j, (a, b) in enumerate(zip(outs[True], outs[False])):
        _same(a, b, f"{kind} step {j}")
    act_ref, rho = oracle.occupancy(sc.points, sc.grid, with_rho=True)
    assert np.array_equal(act, act_ref.astype(np.int64))
    lp = params(True)
    ref = oracle.fuse(act_ref, sc.grid, sc.views, H.oracle_params(lp), n_threads=0,
                      variant="nerf" if lp.variant == 1 else "2dgs", thin_rho=rho if lp.thin else None)
    P, v, c = outs[True][-1]
    rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=f"resident {kind}")
    _say(f"[ok] resident {kind}: {rep}")
