"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: active voxel lists, view bitmasks, segmentation and labels bit-exact
(except counted near-threshold voxels, |P - tau| <= 1e-5, and voxels whose
spatial-gate slack is below 1e-9 relative); float32 P within 1e-5 relative of
the binary64 oracle.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import scenes  # noqa: E402
from tests import _helpers as H  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_case(scene, name, params_kw=None, use_nsamp=False, views=None, points=None, opacity=None, tau_occ=0.5,
             check_labels=True, label_points=None):
    params_kw = params_kw or {}
    views = scene.views if views is None else views
    pts = scene.points if points is None else points
    _say(f"[case] {name}: dim={scene.dim} points={len(pts)} views={len(views)} nsamp={use_nsamp} {params_kw}")
    lp = H.lib_params(scene.voxel, **params_kw)
    op = H.oracle_params(lp)
    ctx, sess = H.make_session(scene, lp, max_views=max(len(views), 1),
                               max_view_pixels=max([v.mask.size for v in views] + [1]), opacity=opacity,
                               tau_occ=tau_occ, points=pts)
    act_gpu = sess.active_indices()
    act_ref = oracle.occupancy(pts, scene.grid, opacity=opacity, tau_occ=tau_occ).astype(np.int64)
    assert np.array_equal(act_gpu, act_ref), f"{name}: active list differs ({len(act_gpu)} vs {len(act_ref)})"
    vs = H.upload_views(views, use_nsamp=use_nsamp)
    res = sess.fuse_views(vs)
    P, v, c = H.fetch(res)
    ref = oracle.fuse(act_ref.astype(np.uint32), scene.grid, views, op, use_nsamp=use_nsamp, n_threads=0)
    rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=name)
    if check_labels:
        lpts = scene.label_points if label_points is None else label_points
        lpts = pts if lpts is None else lpts
        lab_gpu = sess.label_points(H.to_dev(np.asarray(lpts, np.float32).reshape(-1, 3))).cpu().numpy()
        seg_gpu = H.gpu_segmented(P, v, len(act_ref), lp.tau_cons)
        lab_ref = oracle.label(lpts, scene.grid, act_ref[seg_gpu].astype(np.uint32))
        assert np.array_equal(lab_gpu, lab_ref), f"{name}: labels differ"
        lab_orc = oracle.label(lpts, scene.grid, act_ref[ref["seg"].astype(bool)].astype(np.uint32))
        rep["label_mismatch_vs_oracle_seg"] = int((lab_orc != lab_gpu).sum())
    _say(f"[ok] {name}: {rep}")
    sess.close()
    return rep


@pytest.fixture(scope="module")
def c1():
    return scenes.config_scene("c1")


def test_c1_r1(c1):
    rep = run_case(c1, "c1-R1")
    assert rep["n_seg"] > 1000


def test_c1_r2_mask_gate_zero(c1):
    rep = run_case(c1, "c1-R2", dict(mask_gate=0.0))
    assert rep["n_seg"] > 1000


def test_c1_nsamp_footprint_stats(c1):
    run_case(c1, "c1-nsamp", use_nsamp=True)
    run_case(c1, "c1-nsamp-R2", dict(mask_gate=0.0, beta=2.0), use_nsamp=True)


def test_c2_forward_facing_full():
    s = scenes.config_scene("c2")
    rep = run_case(s, "c2-full")
    assert rep["n_seg"] > 100


def test_ragged_and_tiny_sizes():
    s = scenes.make_tiny_sphere(dim=32, n_points=5000, width=127, height=93, focal=90.0, n_views=3)
    run_case(s, "ragged-127x93")
    s2 = scenes.make_tiny_sphere(dim=2, n_points=50, width=9, height=7, focal=6.0, n_views=2)
    run_case(s2, "dim2-9x7", dict(mask_gate=0.0))
    s3 = scenes.make_tiny_sphere(dim=16, n_points=800, width=65, height=1, focal=30.0, n_views=2)
    run_case(s3, "row-65x1", dict(mask_gate=0.0))


def test_empty_and_outside_points(c1):
    run_case(c1, "empty", points=np.zeros((0, 3), np.float32))
    far = np.full((100, 3), 5.0, np.float32)
    far[::3] = np.nan
    run_case(c1, "outside+nan", points=far)


def _adversarial_voxel():
    """A float32 coordinate x0 and a voxel size h = fl(x0 / k0) for which the
    product x0 * fl(1 / h) floors to another integer than the correctly
    rounded quotient x0 / h (found by a seeded search)."""
    rng = np.random.default_rng(11)
    for _ in range(100000):
        x0 = float(np.float32(rng.uniform(0.5, 4.0)))
        k0 = int(rng.integers(3, 60))
        h = x0 / k0
        if np.floor(x0 * (1.0 / h)) != np.floor(x0 / h):
            return x0, k0, h
    raise AssertionError("no adversarial voxel size found")


def test_voxel_floor_is_the_correctly_rounded_division():
    """Points whose coordinates are exact (up to the rounding of the division)
    multiples of the voxel size: the kernels' voxel of a point is
    floor(fl((x - origin) / h)) as in the oracle, also where the faster
    product with fl(1 / h) would floor to the neighbouring voxel."""
    import paper_2601_04860_amd as dv
    x0, k0, h = _adversarial_voxel()
    dim = 512
    coords = [x0 * 2.0 ** m for m in range(4) if k0 * 2 ** m < dim]
    g = np.array(np.meshgrid(coords, coords, coords, indexing="ij"), np.float64).reshape(3, -1).T
    rng = np.random.default_rng(5)
    near = np.nextafter(g.astype(np.float32), np.float32(np.inf))
    other = rng.uniform(0.0, dim * h, (5000, 3))
    pts = np.concatenate([g, near, other]).astype(np.float32)
    grid = dict(origin=(0.0, 0.0, 0.0), voxel=h, dim=dim)
    _say(f"[case] voxel floor: h={h!r} x0={x0!r} k0={k0} points={len(pts)}")
    assert np.floor(np.float64(np.float32(x0)) / h) == k0 - 1 or np.floor(np.float64(np.float32(x0)) / h) == k0
    ctx = dv.Context(0)
    xyz = H.to_dev(pts)
    s = dv.Session(ctx, grid, xyz, params=dv.default_params(h), max_views=1, max_view_pixels=64)
    got = s.active_indices()
    ref = oracle.occupancy(pts, grid).astype(np.int64)
    assert np.array_equal(got, ref), f"active lists differ: {len(got)} vs {len(ref)}"
    s.close()


def test_voxel_index_near_boundaries():
    """Points within 1e-7 .. 1e-3 voxel of voxel boundaries on a grid whose
    voxel size and origin are not powers of two: the float evaluation decides
    only where its error bound keeps it clear of the boundary, the binary64
    one elsewhere; the active list equals the oracle's."""
    import paper_2601_04860_amd as dv
    h, dim = 0.1, 128
    origin = (-3.3, -6.1, -0.7)
    rng = np.random.default_rng(23)
    k = rng.integers(0, dim + 1, (3000, 3)).astype(np.float64)
    delta = rng.choice([-1e-3, -1e-4, -1e-5, -1e-6, -1e-7, 0.0, 1e-7, 1e-6, 1e-5, 1e-4, 1e-3], (3000, 3))
    pts = (np.asarray(origin) + (k + delta) * h).astype(np.float32)
    pts = np.concatenate([pts, np.nextafter(pts, np.float32(np.inf)), np.nextafter(pts, np.float32(-np.inf))])
    grid = dict(origin=origin, voxel=h, dim=dim)
    _say(f"[case] voxel index near boundaries: points={len(pts)}")
    ctx = dv.Context(0)
    s = dv.Session(ctx, grid, H.to_dev(pts), params=dv.default_params(h), max_views=1, max_view_pixels=64)
    got = s.active_indices()
    ref = oracle.occupancy(pts, grid).astype(np.int64)
    assert np.array_equal(got, ref), f"active lists differ: {len(got)} vs {len(ref)}"
    # no fusion yet: the segmentation is empty, every label is 0 (the label kernel shares the voxel index)
    lab = s.label_points(H.to_dev(pts)).cpu().numpy()
    assert not lab.any()
    s.close()


def test_label_paths_alignment_and_tail(c1):
    """Labels through the four-points-per-lane path (aligned buffers) and the
    one-lane path (misaligned xyz or labels, ragged tails) agree with the
    oracle's lookup in the GPU segmentation."""
    import torch
    lp = H.lib_params(c1.voxel)
    ctx, sess = H.make_session(c1, lp)
    act = sess.active_indices()
    P, v, _ = H.fetch(sess.fuse_views(H.upload_views(c1.views)))
    seg = act[H.gpu_segmented(P, v, len(act), lp.tau_cons)].astype(np.uint32)
    pts = np.asarray(c1.label_points, np.float32)
    xyz = H.to_dev(pts)
    cases = [("aligned", xyz, None, 0), ("aligned, n = 4k + 3", xyz[: 4 * (len(pts) // 4 - 1) + 3], None, 0),
             ("xyz off by one point", xyz[1:], None, 1), ("labels off by one byte", xyz[:1001], 1, 0)]
    for name, x, lab_off, p0 in cases:
        n = int(x.shape[0])
        _say(f"[case] labels {name}: n={n}")
        out = None
        if lab_off:
            buf = torch.zeros(n + lab_off, dtype=torch.uint8, device="cuda")
            out = buf[lab_off:]
        got = sess.label_points(x, out).cpu().numpy()
        ref = oracle.label(pts[p0:p0 + n], c1.grid, seg)
        assert np.array_equal(got, ref), name
    sess.close()


def test_rebuild_with_other_point_sets(c1):
    """A session rebuilt with fewer, then more (up to its capacity), then no
    points, then unit-opacity and general-opacity sets in turn, with a fusion
    (a segmentation left in the shared bitfield memory) between the builds,
    gives the oracle's active list every time, and fuses correctly afterwards."""
    import paper_2601_04860_amd as dv
    lp = H.lib_params(c1.voxel)
    pts = np.asarray(c1.points, np.float32)
    rng = np.random.default_rng(17)
    ctx = dv.Context(0)
    xyz0 = H.to_dev(pts[:5000])
    sess = dv.Session(ctx, dict(origin=c1.origin, voxel=c1.voxel, dim=c1.dim), xyz0, params=lp, max_views=4,
                      max_view_pixels=max(v.mask.size for v in c1.views), max_points=len(pts))
    sets = [("5000", pts[:5000], None), ("1234", pts[rng.permutation(len(pts))[:1234]], None),
            ("all", pts, None), ("none", pts[:0], None), ("777", pts[-777:], None),
            ("opacity", pts[:3000], rng.uniform(0.2, 1.0, 3000).astype(np.float32)), ("all again", pts, None)]
    all_dev = H.to_dev(pts)
    sets.insert(-1, ("misaligned xyz (a view one point in)", pts[1:4001], None))  # before the final full set
    for name, p_, op in sets:
        _say(f"[case] rebuild {name}: n={len(p_)}")
        if name.startswith("misaligned"):
            xyz = all_dev[1:4001]
        else:
            xyz = H.to_dev(p_.reshape(-1, 3)) if len(p_) else H.to_dev(np.zeros((0, 3), np.float32))
        opd = None if op is None else H.to_dev(op)
        sess.rebuild(xyz, opacity=opd)
        got = sess.active_indices()
        ref = oracle.occupancy(p_, c1.grid, opacity=op).astype(np.int64)
        assert np.array_equal(got, ref), name
        # leave a segmentation in the session's bitfield before the next build
        # (the bitmap of the next build shares that memory)
        sess.fuse_views(H.upload_views(c1.views))
    P, v, c = H.fetch(sess.fuse_views(H.upload_views(c1.views)))
    ref = oracle.fuse(oracle.occupancy(pts, c1.grid).astype(np.uint32), c1.grid, c1.views, H.oracle_params(lp),
                      n_threads=0)
    H.compare_fusion(P, v, c, ref, lp.tau_cons, where="after rebuilds")
    sess.close()


def test_view_behind_and_out_of_frame(c1):
    away = []
    for v in c1.views:
        cam = dict(v.cam)
        c2w = cam["c2w"].copy()
        c2w[:, 0] *= -1.0
        c2w[:, 2] *= -1.0
        cam["c2w"] = c2w
        away.append(scenes.View(cam=cam, d_cam=v.d_cam, mask=v.mask, dmin=v.dmin, dmed=v.dmed, dmax=v.dmax))
    rep = run_case(c1, "facing-away", views=away)
    assert rep["n_seg"] == 0


def test_general_occupancy_path(c1):
    rng = np.random.default_rng(5)
    op = rng.uniform(0.0, 0.6, size=len(c1.points)).astype(np.float32)
    run_case(c1, "opacity-tau0.5", opacity=op, tau_occ=0.5)
    run_case(c1, "count-tau2", tau_occ=2.0)


def test_sixty_four_views():
    s = scenes.make_tiny_sphere(dim=32, n_points=6000, width=48, height=36, focal=40.0, n_views=64)
    run_case(s, "64-views", dict(mask_gate=0.0))


def test_duplicated_views_and_permutation(c1):
    import paper_2601_04860_amd as dv  # noqa: F401
    lp = H.lib_params(c1.voxel)
    ctx, s = H.make_session(c1, lp, max_views=8)
    vs1 = H.upload_views(c1.views)
    r1 = s.fuse_views(vs1)
    P1, v1, _ = H.fetch(r1)
    vs2 = H.upload_views([c1.views[i] for i in (3, 2, 1, 0)])
    P2, v2, _ = H.fetch(s.fuse_views(vs2))
    assert np.allclose(P1, P2, rtol=1e-6, atol=0)
    perm = {0: 3, 1: 2, 2: 1, 3: 0}
    v1p = np.zeros_like(v1)
    for a, b in perm.items():
        v1p |= ((v1 >> np.uint64(a)) & np.uint64(1)) << np.uint64(b)
    seg1, seg2 = P1 >= 0.5, P2 >= 0.5
    assert np.array_equal(v1p[seg1 & seg2], v2[seg1 & seg2])
    s.close()


def test_determinism_run_twice(c1):
    lp = H.lib_params(c1.voxel, mask_gate=0.0)
    ctx, s = H.make_session(c1, lp)
    vs = H.upload_views(c1.views, use_nsamp=True)
    a = [H.fetch(s.fuse_views(vs)) for _ in range(2)]
    assert a[0][0].tobytes() == a[1][0].tobytes() and a[0][1].tobytes() == a[1][1].tobytes()
    s.close()


def test_repeated_fusion_on_other_streams_and_phase_timing(c1):
    """A second fusion of the same views issues no record upload; on another
    stream it waits for the first upload on the device.  Results equal the
    first fusion bit for bit, and the phase-timing mask times only the
    selected phases (events taken from the kernels' dispatches)."""
    import torch
    lp = H.lib_params(c1.voxel)
    ctx, s = H.make_session(c1, lp)
    vs = H.upload_views(c1.views)
    ref = H.fetch(s.fuse_views(vs))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s.set_timing(phases=("fuse", "cull"))
    s.timings(reset=True)
    for st in (s1, s2, s1):
        _say(f"[case] repeated fusion on stream {st}")
        r = s.alloc_result()
        s.fuse_views(vs, r, stream=st)
        st.synchronize()
        got = H.fetch(r)
        assert got[0].tobytes() == ref[0].tobytes() and got[1].tobytes() == ref[1].tobytes()
        assert np.array_equal(got[2], ref[2])
    t = s.timings(reset=True)
    s.set_timing(False)
    assert t["fuse"][1] == 3 and t["cull"][1] == 3 and t["fuse"][0] > 0.0 and t["cull"][0] > 0.0
    assert t["views"][1] == 0 and t["occupancy"][1] == 0 and t["label"][1] == 0
    s.close()


def test_update_view_append_is_bitwise_full(c1):
    """Folding a new view into the resident binary64 accumulators equals the
    full re-fusion bit for bit; replacing a view re-fuses everything."""
    lp = H.lib_params(c1.voxel, mask_gate=0.0, retain_state=1)
    ctx, s = H.make_session(c1, lp, max_views=8)
    vs = H.upload_views(c1.views)
    n = len(c1.views)
    # fuse the first view, then append the rest one by one
    first = H.upload_views(c1.views[:1])
    s.fuse_views(first)
    for k in range(1, n):
        res = s.update_view(k, vs, k)
    P_inc, v_inc, c_inc = H.fetch(res)
    ctx2, s2 = H.make_session(c1, H.lib_params(c1.voxel, mask_gate=0.0))
    P_full, v_full, c_full = H.fetch(s2.fuse_views(vs))
    assert P_inc.tobytes() == P_full.tobytes()
    assert v_inc.tobytes() == v_full.tobytes()
    assert np.array_equal(c_inc, c_full)
    # replace view 1 by view 3 -> equals fusing [0, 3, 2, 3]
    res = s.update_view(1, vs, 3)
    P_rep, v_rep, _ = H.fetch(res)
    vs4 = H.upload_views([c1.views[i] for i in (0, 3, 2, 3)])
    P_ref, v_ref, _ = H.fetch(s2.fuse_views(vs4))
    assert P_rep.tobytes() == P_ref.tobytes() and v_rep.tobytes() == v_ref.tobytes()
    act = s.active_indices()
    ref = oracle.fuse(act.astype(np.uint32), c1.grid, [c1.views[i] for i in (0, 3, 2, 3)], H.oracle_params(lp))
    H.compare_fusion(P_rep, v_rep, None, ref, lp.tau_cons, where="replace")
    # labels follow the incremental segmentation (bitfield and per-cell counts
    # updated in place across appends and the replace), then a fusion of no
    # views clears them all
    pts = np.asarray(c1.points, np.float32)
    xyz = H.to_dev(pts)
    seg = act[H.gpu_segmented(P_rep, v_rep, len(act), lp.tau_cons)].astype(np.uint32)
    assert np.array_equal(s.label_points(xyz).cpu().numpy(), oracle.label(pts, c1.grid, seg))
    s.fuse_views(H.upload_views([]))
    assert not s.label_points(xyz).cpu().numpy().any()
    s.close()
    s2.close()


@pytest.fixture(scope="module")
def c3():
    s = scenes.config_scene("c3")
    act_ref = oracle.occupancy(s.points, s.grid).astype(np.int64)
    return s, act_ref


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,kw,use_nsamp", [("R1", {}, False), ("R2", dict(mask_gate=0.0), False),
                                               ("R1 n_samp", {}, True), ("R2 n_samp", dict(mask_gate=0.0), True)])
def test_c3_unbounded_full_size(c3, name, kw, use_nsamp):
    """512^3, 3M points, 16 views 1264x832: the active list, every voxel's
    fusion and every point's label against the oracle (all 2.45M voxels, all
    3M points, labels from the oracle's own segmentation).  R2 (mask gate 0)
    sends every in-frame sample through the full thick path, so tau_cons acts;
    n_samp adds the footprint statistics (n_samp sums over each footprint)."""
    s, act_ref = c3
    _say(f"[case] c3 full size {name}: nsamp={use_nsamp} {kw}")
    lp = H.lib_params(s.voxel, **kw)
    op = H.oracle_params(lp)
    ctx, sess = H.make_session(s, lp)
    act = sess.active_indices()
    assert np.array_equal(act, act_ref)
    vs = H.upload_views(s.views, use_nsamp=use_nsamp)
    P, v, c = H.fetch(sess.fuse_views(vs))
    ref = oracle.fuse(act_ref.astype(np.uint32), s.grid, s.views, op, use_nsamp=use_nsamp, n_threads=0)
    rep = H.compare_fusion(P, v, c, ref, lp.tau_cons, where=f"c3 {name}")
    lab = sess.label_points(H.to_dev(s.label_points)).cpu().numpy()
    seg_ref = ref["seg"].astype(bool)
    lab_ref = oracle.label(s.label_points, s.grid, act_ref[seg_ref].astype(np.uint32))
    flagged = (np.abs(ref["P"] - lp.tau_cons) <= 1e-5) | (ref["margin"] < 1e-9)
    if flagged.any():   # points in flagged voxels may differ, the rest may not
        lin = np.array([oracle.point_voxel(p, s.grid) for p in s.label_points[lab != lab_ref]])
        assert np.all(np.isin(lin, act_ref[flagged])), f"c3 {name}: labels differ outside flagged voxels"
    else:
        assert np.array_equal(lab, lab_ref), f"c3 {name}: {int((lab != lab_ref).sum())} labels differ"
    _say(f"[ok] c3 {name}: n_act={len(act)} votes={int(ref['counts'][2])} labelled={int(lab.sum())} {rep}")
    sess.close()
