"""Batched fusion (many sessions, uneven grids and view counts, one persistent
launch sequence, HIP graph replay, autotuned schedule): every item's outputs
equal running it alone, bit for bit, and match the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import scenes  # noqa: E402
from tests import _helpers as H  # noqa: E402


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _scenes():
    out = [scenes.make_tiny_sphere(dim=64, n_points=20000, n_views=4, width=128, height=96, focal=100.0, seed=1),
           scenes.make_tiny_sphere(dim=32, n_points=6000, n_views=6, width=96, height=64, focal=70.0, seed=7),
           scenes.make_tiny_sphere(dim=128, n_points=60000, n_views=3, width=160, height=120, focal=120.0, seed=9),
           scenes.make_forward_facing(dim=128, n_points=80000, n_views=5, width=252, height=189, focal=200.0)]
    return out


@pytest.fixture(scope="module")
def world():
    import paper_2601_04860_amd as dv
    ctx = dv.Context(0)
    items = []
    for k, sc in enumerate(_scenes()):
        for retain in (0, 1):
            lp = dv.default_params(sc.voxel, mask_gate=0.0 if k % 2 else 0.5, retain_state=retain)
            _, sess = H.make_session(sc, lp, ctx=ctx, max_views=len(sc.views) + 2)
            items.append((sc, lp, sess, H.upload_views(sc.views)))
    return ctx, items


def _alone(sc, lp, vs):
    ctx, s = H.make_session(sc, lp, max_views=len(sc.views) + 2)
    out = H.fetch(s.fuse_views(vs))
    s.close()
    return out


@pytest.mark.parametrize("use_graph,schedule", [(False, 0), (True, 0), (False, 1), (True, 4), (True, 16)])
def test_batched_full_fusion_equals_alone(world, use_graph, schedule):
    """schedule 0: a wavefront per chunk from the hardware dispatcher; k > 0:
    the persistent grid pulling k-chunk descriptors from the atomic queue."""
    import paper_2601_04860_amd as dv
    ctx, items = world
    _say(f"[case] batch graph={use_graph} schedule={schedule}")
    b = dv.Batch(ctx, max_items=len(items), max_new_views=64, use_graph=use_graph, schedule=schedule)
    work, res = [], []
    for sc, lp, sess, vs in items:
        r = sess.alloc_result()
        res.append(r)
        work.append((sess, dv.BATCH_FUSE, vs, None, 0, r))
    for rep in range(3):  # replays of the same graph with fresh tables
        b.run(work)
        for (sc, lp, sess, vs), r in zip(items, res):
            P, v, c = H.fetch(r)
            Pa, va, ca = _alone(sc, lp, vs)
            n = sess.info()["n_active"]
            assert P[:n].tobytes() == Pa[:n].tobytes() and v[:n].tobytes() == va[:n].tobytes()
            assert np.array_equal(c, ca)
    # and the oracle agrees
    sc, lp, sess, vs = items[3]
    act = sess.active_indices()
    ref = oracle.fuse(act.astype(np.uint32), sc.grid, sc.views, H.oracle_params(lp))
    P, v, c = H.fetch(res[3])
    H.compare_fusion(P, v, c, ref, lp.tau_cons, where="batch-item3")
    b.close()


def test_batch_grows_and_changes_kernel(world):
    """One batch object runs a small batch, then a larger one (its captured
    launch is too small and is rebuilt), then a batch whose views carry n_samp
    (the generic kernel, no graph), then the small one again; every run equals
    the items alone."""
    import paper_2601_04860_amd as dv
    ctx, items = world
    b = dv.Batch(ctx, max_items=len(items), max_new_views=64, use_graph=True)
    small = items[1:3]
    plans = [("small", small, False), ("all", items, False), ("small", small, False)]
    for name, its, _ in plans:
        work, res = [], []
        for sc, lp, sess, vs in its:
            r = sess.alloc_result()
            res.append(r)
            work.append((sess, dv.BATCH_FUSE, vs, None, 0, r))
        _say(f"[case] batch {name}: {len(work)} items")
        b.run(work)
        for (sc, lp, sess, vs), r in zip(its, res):
            P, v, c = H.fetch(r)
            Pa, va, ca = _alone(sc, lp, vs)
            n = sess.info()["n_active"]
            assert P[:n].tobytes() == Pa[:n].tobytes() and v[:n].tobytes() == va[:n].tobytes(), name
            assert np.array_equal(c, ca), name
    # n_samp views: the generic fusion kernel
    sc, lp, sess, _ = items[0]
    vs_ns = H.upload_views(sc.views, use_nsamp=True)
    r = sess.alloc_result()
    b.run([(sess, dv.BATCH_FUSE, vs_ns, None, 0, r)])
    P, v, c = H.fetch(r)
    ctx2, s2 = H.make_session(sc, lp, max_views=len(sc.views) + 2)
    Pa, va, ca = H.fetch(s2.fuse_views(vs_ns))
    n = sess.info()["n_active"]
    assert P[:n].tobytes() == Pa[:n].tobytes() and v[:n].tobytes() == va[:n].tobytes()
    s2.close()
    b.close()


def test_batched_updates_equal_sequential(world):
    """A batch of one-view updates (fold for retaining sessions, full re-fusion
    otherwise) equals the same updates issued one session at a time."""
    import paper_2601_04860_amd as dv
    ctx, items = world
    b = dv.Batch(ctx, max_items=len(items), max_new_views=len(items), schedule=4)
    # start every session from its first two views
    for sc, lp, sess, vs in items:
        first = H.upload_views(sc.views[:2])
        sess.fuse_views(first)
        sess._first = first
    work, res = [], []
    for sc, lp, sess, vs in items:
        r = sess.alloc_result()
        res.append(r)
        work.append((sess, dv.BATCH_UPDATE, vs, 2, 2, r))
    b.run(work)
    for (sc, lp, sess, vs), r in zip(items, res):
        P, v, c = H.fetch(r)
        Pa, va, ca = _alone(sc, lp, H.upload_views(sc.views[:3]))
        n = sess.info()["n_active"]
        assert P[:n].tobytes() == Pa[:n].tobytes(), sc.name
        assert v[:n].tobytes() == va[:n].tobytes()
    b.close()


def test_autotune_and_cache(world, tmp_path):
    import paper_2601_04860_amd as dv
    ctx, items = world
    b = dv.Batch(ctx, max_items=len(items), max_new_views=64)
    work = [(sess, dv.BATCH_FUSE, vs, None, 0, sess.alloc_result()) for sc, lp, sess, vs in items]
    path = tmp_path / "tune.jsonl"
    cfg = b.tune(work, cache_path=path)
    _say(f"[ok] tuned {cfg}")
    assert path.exists() and cfg["fuse_waves_per_block"] in (1, 2, 4, 8) and cfg["cull_blocks_per_cu"] in (2, 4, 8)
    assert cfg["schedule"] in (0, 1, 4, 16) and cfg["use_graph"] in (0, 1)
    cfg2 = b.tune(work, cache_path=path)  # served from the cache
    assert cfg2 == cfg
    b.run(work)
    for (sc, lp, sess, vs), w in zip(items, work):
        P, v, c = H.fetch(w[5])
        Pa, va, ca = _alone(sc, lp, vs)
        n = sess.info()["n_active"]
        assert P[:n].tobytes() == Pa[:n].tobytes()
    b.close()


def test_batch_rejects_bad_items(world):
    import paper_2601_04860_amd as dv
    ctx, items = world
    b = dv.Batch(ctx, max_items=2, max_new_views=8)
    sc, lp, sess, vs = items[0]
    r = sess.alloc_result()
    with pytest.raises(dv.DivasError) as e:
        b.run([(sess, dv.BATCH_FUSE, vs, None, 0, r), (sess, dv.BATCH_FUSE, vs, None, 0, r)])
    assert e.value.status == dv.ERR_ARG
    with pytest.raises(dv.DivasError) as e:
        b.run([(s, dv.BATCH_FUSE, v, None, 0, s.alloc_result()) for _, _, s, v in items[:3]])
    assert e.value.status == dv.ERR_CAPACITY
    b.close()
