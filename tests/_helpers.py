"""Shared helpers of the GPU parity tests: upload a synthetic scene to the
device, run the library through its C ABI, and compare with the oracle."""
from __future__ import annotations

import numpy as np



def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def upload_views(views, use_nsamp=False, use_logit=False):
    import torch
    import paper_2601_04860_amd as dv
    vs = dv.ViewSet()
    for v in views:
        mask = v.logit if use_logit else v.mask
        ns = None
        if use_nsamp and v.nsamp is not None:
            ns = to_dev(v.nsamp.view(np.int16))  # uint16 bits carried in an int16 tensor
        vs.add(v.cam, v.d_cam, to_dev(mask), to_dev(v.dmin), to_dev(v.dmed), to_dev(v.dmax), ns)
    return vs


def make_session(scene, params, max_views=None, max_view_pixels=None, ctx=None, opacity=None, tau_occ=0.5,
                 points=None):
    import paper_2601_04860_amd as dv
    ctx = ctx or dv.Context(0)
    pts = scene.points if points is None else points
    xyz = to_dev(np.asarray(pts, np.float32).reshape(-1, 3))
    op = None if opacity is None else to_dev(np.asarray(opacity, np.float32))
    mv = max_views or max(len(scene.views), 1)
    mp = max_view_pixels or max([v.mask.size for v in scene.views] + [1])
    s = dv.Session(ctx, dict(origin=scene.origin, voxel=scene.voxel, dim=scene.dim), xyz, opacity=op,
                   tau_occ=tau_occ, params=params, max_views=mv, max_view_pixels=mp)
    s._keep_xyz = (xyz, op)
    return ctx, s


def lib_params(voxel, **kw):
    import paper_2601_04860_amd as dv
    return dv.default_params(voxel, **kw)


def oracle_params(lp):
    return dict(gamma=lp.gamma, beta=lp.beta, gamma_st=lp.gamma_st, alpha1=lp.alpha1, k_grad=lp.k_grad, eps=lp.eps,
                tau_cons=lp.tau_cons, mask_gate=lp.mask_gate, soft_width=lp.soft_width,
                lambda_range=lp.lambda_range, b_max=lp.b_max, rho_thin=lp.rho_thin, tau_thin=lp.tau_thin,
                rho_cover=lp.rho_cover, rho_occ=lp.rho_occ, n_abs=lp.n_abs,
                nerf_ray_depths=bool(lp.nerf_ray_depths))


def fetch(res):
    import torch
    torch.cuda.synchronize()
    P = res["P"].cpu().numpy()
    v = res["vmask"].cpu().numpy().view(np.uint64)
    c = res["counts"].cpu().numpy() if res.get("counts") is not None else None
    return P, v, c


def popcount(u64):
    """Total number of set bits of a uint64 array."""
    a = np.ascontiguousarray(u64, dtype=np.uint64)
    return int(np.unpackbits(a.view(np.uint8)).sum())


def gpu_segmented(P_gpu, v_gpu, n, tau_cons):
    """The device's segmentation of the first n voxels: its binary64 decision
    P >= tau, read from the vote mask it writes for segmented voxels only
    (nonzero there once tau > 0), since the float32 P can round a voxel within
    1e-5 of tau onto the other side."""
    if tau_cons > 0:
        return np.asarray(v_gpu[:n]) != 0
    return np.asarray(P_gpu[:n]).astype(np.float64) >= tau_cons


def compare_fusion(P_gpu, v_gpu, counts_gpu, ref, tau_cons, where=""):
    """The parity bar: float32 P within 1e-5 relative of the binary64 oracle,
    view bitmasks and segmentation bit-exact except for counted near-threshold
    voxels (|P - tau| <= 1e-5) and voxels whose spatial-gate slack is below
    1e-9 relative (decision margin).  Returns a small report dict."""
    n = len(ref["P"])
    assert len(P_gpu) >= n, where
    P_gpu = P_gpu[:n]
    v_gpu = v_gpu[:n]
    Pr = ref["P"]
    flag_thr = np.abs(Pr - tau_cons) <= 1e-5
    flag_margin = ref["margin"] < 1e-9
    # values
    zero = Pr == 0
    assert np.all(P_gpu[zero] == 0), f"{where}: nonzero P where the oracle has 0"
    rel = np.abs(P_gpu[~zero].astype(np.float64) - Pr[~zero]) / np.abs(Pr[~zero])
    bad_val = np.zeros(n, bool)
    bad_val[~zero] = rel > 1e-5
    # decisions
    seg_gpu = P_gpu.astype(np.float64) >= tau_cons
    bad_vraw = (v_gpu != ref["vout"])
    bad_seg = seg_gpu != ref["seg"].astype(bool)
    allowed = flag_thr | flag_margin
    unexplained = (bad_val | bad_vraw | bad_seg) & ~allowed
    rep = dict(n=n, n_seg=int(ref["seg"].sum()), n_flag_thr=int(flag_thr.sum()), n_flag_margin=int(flag_margin.sum()),
               n_mismatch=int((bad_val | bad_vraw | bad_seg).sum()), max_rel=float(rel.max()) if rel.size else 0.0)
    assert not unexplained.any(), f"{where}: {int(unexplained.sum())} unexplained mismatches, first " \
                                  f"{np.flatnonzero(unexplained)[:5]}; report {rep}"
    if counts_gpu is not None:
        # the count is of binary64 decisions P >= tau; a voxel within 1e-5 of
        # tau may round onto the other side in the float32 output
        assert abs(int(counts_gpu[0]) - int(seg_gpu.sum())) <= int(flag_thr.sum()), where
        assert counts_gpu[0] == int(ref["seg"].sum()) or flag_thr.any() or flag_margin.any(), where
        assert counts_gpu[2] == popcount(ref["vraw"]) or flag_margin.any(), where
        assert counts_gpu[1] == int(flag_thr.sum()), where
    return rep
