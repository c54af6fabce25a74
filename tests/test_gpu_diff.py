"""GPU parity of the differentiable fusion and its hand-written adjoint
(torch.autograd.Function) against the binary64 oracle: forward P, gradients
w.r.t. logits and depth maps, FP64 finite differences, determinism."""
import math
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


@pytest.fixture(scope="module")
def c4():
    s = scenes.config_scene("c4")
    g = s.dim
    act = oracle.occupancy(s.points, s.grid).astype(np.int64)
    ijk = np.stack([act % g, (act // g) % g, act // (g * g)], 1)
    crop = np.all(ijk >= g // 2, 1)  # a 32^3 crop (positive octant) holding sphere surface
    rng = np.random.default_rng(44)
    coef = np.where(crop, rng.normal(size=len(act)), 0.0)
    return s, act, coef


def _session(s):
    import paper_2601_04860_amd as dv
    lp = dv.default_params(s.voxel, differentiable=1, mask_gate=0.0, soft_width=0.01)
    ctx, sess = H.make_session(s, lp)
    return lp, sess


def _torch_maps(s):
    import torch
    L = [H.to_dev(v.logit).requires_grad_(True) for v in s.views]
    Dn = [H.to_dev(v.dmin).requires_grad_(True) for v in s.views]
    Dm = [H.to_dev(v.dmed).requires_grad_(True) for v in s.views]
    Dx = [H.to_dev(v.dmax).requires_grad_(True) for v in s.views]
    cams = [(v.cam, v.d_cam) for v in s.views]
    return cams, L, Dn, Dm, Dx, torch


def _forward_and_adjoint(s, act, coef, name, min_nnz):
    _say(f"[case] {name} diff: n_act={len(act)} weighted={int((coef != 0).sum())}")
    from paper_2601_04860_amd.autograd import fused_scores
    lp, sess = _session(s)
    assert np.array_equal(sess.active_indices(), act)
    cams, L, Dn, Dm, Dx, torch = _torch_maps(s)
    P = fused_scores(sess, cams, L, Dn, Dm, Dx)
    op = H.oracle_params(lp)
    P_ref, _, _ = oracle.fuse_diff(act.astype(np.uint32), s.grid, s.views, op)
    Pg = P.detach().cpu().numpy().astype(np.float64)
    # background logits reach -400: P ~ 1e-174 in binary64 underflows the float32 output
    P32 = P_ref.astype(np.float32).astype(np.float64)
    bad = Pg != P32
    assert np.array_equal(Pg == 0, P32 == 0), np.flatnonzero((Pg == 0) != (P32 == 0))[:10]
    nz = np.abs(P_ref) > 1e-30
    assert np.max(np.abs(Pg[nz] - P_ref[nz]) / np.abs(P_ref[nz])) <= 1e-5
    _say(f"[ok] {name} forward: nonzero={int(nz.sum())} differing-from-float32(oracle)={int(bad.sum())}")
    loss = (P.double() * torch.from_numpy(coef).to(P.device)).sum()
    loss.backward()
    g_ref = oracle.fuse_diff_grad(act.astype(np.uint32), s.grid, s.views, op, coef)
    stats = {}
    for key, ts in (("logit", L), ("dmin", Dn), ("dmed", Dm), ("dmax", Dx)):
        gmax = max(np.abs(g).max() for g in g_ref[key])
        nnz = 0
        for t, gr in zip(ts, g_ref[key]):
            gg = t.grad.cpu().numpy().astype(np.float64)
            err = np.abs(gg - gr)
            assert np.all(err <= 1e-5 * np.abs(gr) + 1e-6 * gmax), (key, float(err.max()), gmax)
            nnz += np.count_nonzero(gr)
        assert nnz > min_nnz[key], (key, nnz)
        stats[key] = (gmax, nnz)
        _say(f"[ok] {name} grad {key}: max|g|={gmax:.3e} nonzero={nnz}")
    sess.close()
    return stats


def test_diff_forward_and_adjoint_match_oracle(c4):
    s, act, coef = c4
    _forward_and_adjoint(s, act, coef, "c4", dict(logit=10, dmin=10, dmed=10, dmax=10))


def _finite_differences(s, act, coef, name, per_view, rng=None):
    """GPU gradient vs central differences of the binary64 forward at the
    largest-gradient pixels and (with rng) at random pixels with a nonzero
    gradient; perturbations exact in float32; pixels where a hard gate flips
    inside the step are skipped."""
    import paper_2601_04860_amd as dv  # noqa: F401
    lp, sess = _session(s)
    cams, L, Dn, Dm, Dx, torch = _torch_maps(s)
    from paper_2601_04860_amd.autograd import fused_scores
    P = fused_scores(sess, cams, L, Dn, Dm, Dx)
    (P.double() * torch.from_numpy(coef).to(P.device)).sum().backward()
    op = H.oracle_params(lp)
    P0 = oracle.fuse_diff(act.astype(np.uint32), s.grid, s.views, op)[0]
    checked = 0
    for key, ts, step in (("logit", L, 2.0 ** -8), ("dmin", Dn, 2.0 ** -14), ("dmed", Dm, 2.0 ** -14),
                          ("dmax", Dx, 2.0 ** -14)):
        grads = [t.grad.cpu().numpy().astype(np.float64) for t in ts]
        gmax = max(np.abs(g).max() for g in grads)
        for si, g in enumerate(grads):
            picks = list(np.argsort(-np.abs(g).ravel())[:per_view])
            if rng is not None:
                nzp = np.flatnonzero(np.abs(g).ravel() > 1e-3 * gmax)
                picks += list(rng.choice(nzp, size=min(per_view, len(nzp)), replace=False))
            for flat in picks:
                y, x = np.unravel_index(flat, g.shape)
                if abs(g[y, x]) <= 1e-3 * gmax:
                    continue
                vals = []
                for sg in (1, -1):
                    vv = list(s.views)
                    v = vv[si]
                    arr = getattr(v, key).copy()
                    arr[y, x] = np.float32(float(arr[y, x]) + sg * step)
                    d = dict(cam=v.cam, d_cam=v.d_cam, mask=v.mask, dmin=v.dmin, dmed=v.dmed, dmax=v.dmax,
                             logit=v.logit)
                    d[key] = arr
                    vv[si] = scenes.View(**d)
                    vals.append(float(np.dot(coef, oracle.fuse_diff(act.astype(np.uint32), s.grid, vv, op)[0] - P0)))
                fwd, bwd = vals[0] / step, -vals[1] / step
                if abs(fwd - bwd) > 0.05 * (abs(fwd) + abs(bwd) + 1e-30):
                    continue  # kink of a hard gate inside the step
                fd = (vals[0] - vals[1]) / (2 * step)
                assert math.isclose(fd, g[y, x], rel_tol=1e-4, abs_tol=1e-6 * gmax + 6e-16 / step), (key, si, y, x)
                checked += 1
    _say(f"[ok] {name} finite differences: {checked} entries")
    sess.close()
    return checked


def test_adjoint_against_fp64_finite_differences(c4):
    s, act, coef = c4
    assert _finite_differences(s, act, coef, "c4", 3) >= 10


@pytest.fixture(scope="module")
def c4u():
    """The differentiable workload with unsaturated logits (0.5 * signed pixel
    distance + N(0, 0.2)), the loss weighting every active voxel, and d_cam = 2
    so that far pixels are see-through (front reference)."""
    s = scenes.config_scene("c4", slope=0.5)
    for v in s.views:
        v.d_cam = 2.0
    act = oracle.occupancy(s.points, s.grid).astype(np.int64)
    coef = np.random.default_rng(45).normal(size=len(act))
    return s, act, coef


def test_unsaturated_adjoint_exercises_every_branch(c4u):
    """Thousands of votes carry gradient; the lower and upper clamps of t and
    the front (see-through) reference all occur among them, and the adjoint
    matches the oracle's exact gradient there."""
    s, act, coef = c4u
    import paper_2601_04860_amd as dv
    lp = dv.default_params(s.voxel, differentiable=1, mask_gate=0.0, soft_width=0.01)
    br = oracle.fuse_diff_branches(act.astype(np.uint32), s.grid, s.views, H.oracle_params(lp), coef)
    _say(f"[case] c4 unsaturated branches: {br}")
    assert br["votes"] > 3000 and br["lo_clamp"] > 500 and br["hi_clamp"] > 500 and br["front"] > 100
    st = _forward_and_adjoint(s, act, coef, "c4u", dict(logit=3000, dmin=500, dmed=500, dmax=500))
    assert st["logit"][0] > 1e-2 and st["dmin"][0] > 1e-2


def test_unsaturated_adjoint_against_finite_differences(c4u):
    s, act, coef = c4u
    assert _finite_differences(s, act, coef, "c4u", 3, rng=np.random.default_rng(46)) >= 40


def test_adjoint_is_deterministic(c4):
    s, act, coef = c4
    lp, sess = _session(s)
    import torch
    vs = H.upload_views(s.views, use_logit=True)
    sess.fuse_views(vs)
    g = torch.from_numpy(coef.astype(np.float32)).cuda()
    outs = []
    for _ in range(2):
        grads = {k: [torch.empty(v.dmed.shape, dtype=torch.float32, device="cuda") for v in s.views]
                 for k in ("logit", "dmin", "dref", "dmax")}
        sess.fuse_backward(g, grads)
        torch.cuda.synchronize()
        outs.append(b"".join(t.cpu().numpy().tobytes() for k in grads for t in grads[k]))
    assert outs[0] == outs[1]
    sess.close()


def test_soft_width_limit_equals_hard_R2(c4):
    """As w_s -> 0 the differentiable forward equals the hard thick path with
    mask_gate = 0 on m = sigmoid(logit) (no n_samp)."""
    s, act, coef = c4
    import paper_2601_04860_amd as dv
    lp = dv.default_params(s.voxel, differentiable=1, mask_gate=0.0, soft_width=1e-12)
    ctx, sess = H.make_session(s, lp)
    P, _, _ = H.fetch(sess.fuse_views(H.upload_views(s.views, use_logit=True)))
    hard = [scenes.View(cam=v.cam, d_cam=v.d_cam,
                        mask=(1 / (1 + np.exp(-v.logit.astype(np.float64)))).astype(np.float32),
                        dmin=v.dmin, dmed=v.dmed, dmax=v.dmax) for v in s.views]
    lp2 = dv.default_params(s.voxel, mask_gate=0.0)
    ctx2, s2 = H.make_session(s, lp2)
    P2, _, _ = H.fetch(s2.fuse_views(H.upload_views(hard)))
    n = len(act)
    assert np.array_equal(P[:n] > 0, P2[:n] > 0)
    assert np.allclose(P[:n], P2[:n], rtol=1e-6, atol=1e-7)
    sess.close()
    s2.close()


def test_stale_forward_and_view_count_are_refused(c4):
    """A forward whose session was fused again before .backward() raises
    instead of returning the gradient of the newer fusion; the adjoint call
    refuses gradient arrays for another number of views."""
    import torch

    import paper_2601_04860_amd as dv
    from paper_2601_04860_amd.autograd import fused_scores
    s, act, coef = c4
    _say("[case] stale forward and view count")
    lp, sess = _session(s)
    cams, L, Dn, Dm, Dx, torch = _torch_maps(s)
    P = fused_scores(sess, cams, L, Dn, Dm, Dx)
    P2 = fused_scores(sess, cams[:2], L[:2], Dn[:2], Dm[:2], Dx[:2])  # fuses the session again
    with pytest.raises(RuntimeError, match="fused or updated again"):
        P.sum().backward()
    P2.sum().backward()  # the latest forward still differentiates
    assert L[0].grad is not None and L[2].grad is None
    n = sess.info()["n_active"]
    g = torch.zeros(max(n, 1), dtype=torch.float32, device="cuda")
    grads = [torch.empty_like(L[0]) for _ in range(3)]
    ptrs = (dv.C.c_void_p * 3)(*[t.data_ptr() for t in grads])
    st = dv._lib.divas_fuse_backward(sess._h, g.data_ptr(), 3, dv.C.cast(ptrs, dv.C.c_void_p), None, None, None, None)
    assert st == dv.ERR_ARG
    sess.close()
