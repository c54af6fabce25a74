"""CPU oracle for depth-weighted voxel aggregation -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C (``divas_oracle.c``) behind ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the HIP library and its Python binding never do, and the two
share no code.

Every function restates a passage of the paper (DivAS, arXiv 2601.04860):
  occupancy()  -- active-voxel list of the 2DGS occupancy construction
                  (Sec. 3.5 "Occupancy by Morton-scattered opacity", App. F)
  fuse()       -- thick path of Alg. gs-fusion, Eq. compact-fusion; with
                  thin_rho the thin fallback (Alg. gs-thin); variant "nerf"
                  Alg. nerf-fusion (and Alg. nerf-thin with thin_rho)
  label()      -- Eq. pass1 (Pass 1 of Alg. vox2surfel)
  surfel_coverage() -- Pass 3 of Alg. vox2surfel (footprint coverage, kappa)
  fuse_diff(), fuse_diff_grad() -- the differentiable variant (soft depth
                  test on logits) and its exact gradient; not in the paper.
  pi_dg_map()  -- App. D depth-gradient factor.

Pins: tests/test_oracle_*pins.py check these functions against closed forms,
brute force and invariants, and tests/test_oracle_mutations.py checks that
planted mistakes fail them; the end-to-end fused values on the synthetic
scenes are "parity unpinned" by the paper (it prints no worked example).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "divas_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A mutation check may point the tests at a deliberately broken build of the
# oracle (planted mistakes live on the CPU only).
_LIB_OVERRIDE = os.environ.get("DIVAS_ORACLE_LIB")
_lib = None


def build(force=True):
    """Compile the oracle with gcc: binary64, no FP contraction, OpenMP."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OCam(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("c2w", C.c_double * 12), ("width", C.c_int32), ("height", C.c_int32),
                ("d_cam", C.c_double)]


class OParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("gamma", "beta", "gamma_st", "alpha1", "k_grad", "eps",
                                          "tau_cons", "mask_gate", "soft_width")]


class OMaps(C.Structure):
    _fields_ = [("mask", C.c_void_p), ("dmin", C.c_void_p), ("dmed", C.c_void_p),
                ("dmax", C.c_void_p), ("nsamp", C.c_void_p)]


class ONerf(C.Structure):
    _fields_ = [("lambda_range", C.c_double), ("b_max", C.c_double), ("ray_depths", C.c_int),
                ("thin", C.c_int), ("rho_thin", C.c_double), ("tau_thin", C.c_double), ("rho_cover", C.c_double)]


class OResult(C.Structure):
    _fields_ = [("P", C.c_void_p), ("W", C.c_void_p), ("Z", C.c_void_p), ("vraw", C.c_void_p),
                ("vout", C.c_void_p), ("seg", C.c_void_p), ("margin", C.c_void_p),
                ("counts", C.c_int64 * 3)]


def lib():
    global _lib
    if _lib is None and _LIB_OVERRIDE:
        _lib = _declare(C.CDLL(_LIB_OVERRIDE))
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(C.CDLL(_LIB_PATH))
    return _lib


def _declare(L):
    if True:
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.oracle_occupancy.argtypes = [vp, vp, i64, vp, dbl, i32, dbl, vp, vp]
        L.oracle_occupancy.restype = i64
        L.oracle_fuse.argtypes = [vp, i64, vp, dbl, i32, i32, vp, vp, vp, C.c_int, vp]
        L.oracle_fuse_nerf.argtypes = [vp, i64, vp, dbl, i32, i32, vp, vp, vp, vp, vp, C.c_int, vp]
        L.oracle_surfel_coverage.argtypes = [vp, vp, vp, i64, vp, vp, dbl, i32, vp, i64, vp, i32, vp, vp, dbl, dbl,
                                             dbl, vp, vp]
        L.oracle_surfel_coverage.restype = i64
        L.oracle_surfel_view_counts.argtypes = [vp, vp, dbl, dbl, vp, vp, vp, vp, vp]
        L.oracle_surfel_view_counts.restype = C.c_int
        L.oracle_fuse_thin.argtypes = [vp, i64, vp, dbl, i32, i32, vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl,
                                       C.c_int, vp]
        L.oracle_label.argtypes = [vp, i64, vp, dbl, i32, vp, i64, vp]
        L.oracle_fuse_diff.argtypes = [vp, i64, vp, dbl, i32, i32, vp, vp, vp, vp, vp, vp]
        L.oracle_fuse_diff_grad.argtypes = [vp, i64, vp, dbl, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_pi_dg_map.argtypes = [vp, vp, C.c_int, C.c_int, dbl, vp]
        L.oracle_fuse_diff_branches.argtypes = [vp, i64, vp, dbl, i32, i32, vp, vp, vp, vp, vp]
        L.oracle_project.argtypes = [vp, vp, dbl, vp, vp, vp]
        L.oracle_project.restype = C.c_int
        L.oracle_pixel_ray.argtypes = [vp, C.c_int, C.c_int, vp, vp]
        L.oracle_footprint_stats.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                             C.c_uint16, vp, vp]
        L.oracle_morton3.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_morton3.restype = C.c_uint64
        L.oracle_point_voxel.argtypes = [vp, vp, dbl, i32]
        L.oracle_point_voxel.restype = i64
        L.oracle_num_threads.restype = C.c_int
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_params(voxel, **kw):
    """Defaults of Tab. gs-hyperparams; alpha1, k and eps are not given by the
    paper (readings: alpha1 = 1, k = 1/(4 h^2), eps = 1e-6)."""
    p = dict(gamma=1.0, beta=0.05, gamma_st=1.5, alpha1=1.0, k_grad=1.0 / (4.0 * voxel * voxel),
             eps=1e-6, tau_cons=0.5, mask_gate=0.5, soft_width=0.01)
    p.update({k: v for k, v in kw.items() if v is not None})
    return p


def _oparams(p):
    return OParams(**{k: float(p[k]) for k in ("gamma", "beta", "gamma_st", "alpha1", "k_grad", "eps",
                                                "tau_cons", "mask_gate", "soft_width")})


def _ocam(v):
    cam = v.cam if hasattr(v, "cam") else v
    c = OCam()
    c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    flat = np.asarray(cam["c2w"], np.float64).reshape(12)
    for i in range(12):
        c.c2w[i] = float(flat[i])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.d_cam = float(getattr(v, "d_cam", cam.get("d_cam", 0.0)) if hasattr(v, "cam") else cam.get("d_cam", 0.0))
    return c


class _ViewPack:
    """Keeps contiguous copies alive while the C code reads them."""

    def __init__(self, views, use_nsamp, use_logit=False):
        n = len(views)
        self.cams = (OCam * max(n, 1))()
        self.maps = (OMaps * max(n, 1))()
        self.keep = []
        for i, v in enumerate(views):
            self.cams[i] = _ocam(v)
            src = v.logit if use_logit else v.mask
            arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (src, v.dmin, v.dmed, v.dmax)]
            ns = np.ascontiguousarray(v.nsamp, dtype=np.uint16) if (use_nsamp and v.nsamp is not None) else None
            self.keep += arrs + [ns]
            self.maps[i] = OMaps(_p(arrs[0]).value, _p(arrs[1]).value, _p(arrs[2]).value,
                                 _p(arrs[3]).value, None if ns is None else _p(ns).value)


def occupancy(points, grid, opacity=None, tau_occ=0.5, with_rho=False):
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    n = len(pts)
    out = np.zeros(max(n, 1), np.uint32)
    rho = np.zeros(max(n, 1), np.float64) if with_rho else None
    op = None if opacity is None else np.ascontiguousarray(opacity, dtype=np.float32)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    na = lib().oracle_occupancy(_p(pts), _p(op), n, _p(origin), float(grid["voxel"]), int(grid["dim"]),
                                float(tau_occ), _p(out), _p(rho))
    if with_rho:
        return out[:na].copy(), rho[:na].copy()
    return out[:na].copy()


def nerf_default_params(voxel, scenes_kind="360", **kw):
    """NeRF constants of the NeRF hyperparameter table (LLFF / Mip-NeRF 360
    columns): gamma, beta, b_max, lambda_range and, for the thin path,
    rho_thin (thin_density_thresh), rho_cover (thin_percent_cover) and
    tau_thin; the remaining constants as default_params.  nerf_ray_depths
    False (default) reads the depth tuple as camera Z, as the paper states for
    both renderers; True reads it as distances along the pixel rays."""
    col = {"llff": dict(gamma=4.0, beta=0.2, b_max=10.0, lambda_range=0.05, rho_thin=50.0, rho_cover=0.2),
           "360": dict(gamma=0.5, beta=0.2, b_max=1.0, lambda_range=5.0, rho_thin=30.0, rho_cover=0.3)}[scenes_kind]
    p = default_params(voxel)
    p.update(col)
    p.update(tau_thin=0.6, nerf_ray_depths=False)
    p.update({k: v for k, v in kw.items() if v is not None})
    return p


# 2DGS thin path: the paper keeps no separate thin density floor for 2DGS; the
# eligibility test uses the thick path's floor rho_thresh = 0.5.
THIN_DEFAULTS = dict(rho_thin=0.5, tau_thin=0.6, rho_cover=0.5, rho_occ=0.1, n_abs=25.0)


def fuse(active, grid, views, params, use_nsamp=False, n_threads=1, with_margin=True, variant="2dgs",
         thin_rho=None):
    """Returns a dict of per-voxel arrays: P (f64), W, Z, vraw, vout (u64), seg (u8),
    margin (f64) and counts (n_seg, n_threshold_flagged, n_votes).
    variant "nerf": the NeRF path of Alg. nerf-fusion (params carry
    lambda_range, b_max and nerf_ray_depths); with thin_rho it adds the thin
    path of Alg. nerf-thin (params carry rho_thin, tau_thin, rho_cover).
    thin_rho (float64 per active voxel) without variant "nerf": the 2DGS path
    with the thin-structure fallback of Alg. gs-thin (params carry rho_thin,
    tau_thin, rho_cover, rho_occ, n_abs; THIN_DEFAULTS otherwise)."""
    act = np.ascontiguousarray(active, dtype=np.uint32)
    n = len(act)
    res = {k: np.zeros(max(n, 1), np.float64) for k in ("P", "W", "Z", "margin")}
    res["vraw"] = np.zeros(max(n, 1), np.uint64)
    res["vout"] = np.zeros(max(n, 1), np.uint64)
    res["seg"] = np.zeros(max(n, 1), np.uint8)
    r = OResult(_p(res["P"]).value, _p(res["W"]).value, _p(res["Z"]).value, _p(res["vraw"]).value,
                _p(res["vout"]).value, _p(res["seg"]).value,
                _p(res["margin"]).value if with_margin else None)
    vp = _ViewPack(views, use_nsamp)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    pr = _oparams(params)
    if variant == "nerf":
        rho = None if thin_rho is None else np.ascontiguousarray(thin_rho, dtype=np.float64)
        nr = ONerf(float(params["lambda_range"]), float(params["b_max"]),
                   1 if params.get("nerf_ray_depths", False) else 0, 0 if rho is None else 1,
                   float(params.get("rho_thin", 30.0)), float(params.get("tau_thin", 0.6)),
                   float(params.get("rho_cover", 0.3)))
        lib().oracle_fuse_nerf(_p(act), n, _p(origin), float(grid["voxel"]), int(grid["dim"]), len(views),
                               C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p), C.byref(pr), C.byref(nr),
                               _p(rho), int(n_threads), C.byref(r))
    elif thin_rho is not None:
        rho = np.ascontiguousarray(thin_rho, dtype=np.float64)
        tp = {k: float(params.get(k, v)) for k, v in THIN_DEFAULTS.items()}
        lib().oracle_fuse_thin(_p(act), n, _p(origin), float(grid["voxel"]), int(grid["dim"]), len(views),
                               C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p), C.byref(pr), _p(rho),
                               tp["rho_thin"], tp["tau_thin"], tp["rho_cover"], tp["rho_occ"], tp["n_abs"],
                               int(n_threads), C.byref(r))
    else:
        lib().oracle_fuse(_p(act), n, _p(origin), float(grid["voxel"]), int(grid["dim"]), len(views),
                          C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p), C.byref(pr),
                          int(n_threads), C.byref(r))
    out = {k: v[:n].copy() for k, v in res.items()}
    out["counts"] = np.array(list(r.counts), np.int64)
    return out


def surfel_coverage(xyz, scales, quats, labels_in, grid, active, vmask, views, tau_M=0.5, tau_kappa=0.5,
                    eps=1e-6):
    """Pass 3 of Alg. vox2surfel: returns (kappa float64 [n], labels uint8 [n])."""
    pts = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    n = len(pts)
    sc = np.ascontiguousarray(scales, np.float32).reshape(-1, 2)
    qs = np.ascontiguousarray(quats, np.float32).reshape(-1, 4)
    li = np.ascontiguousarray(labels_in, np.uint8)
    act = np.ascontiguousarray(active, np.uint32)
    vm = np.ascontiguousarray(vmask, np.uint64)
    assert len(sc) == n and len(qs) == n and len(li) == n and len(vm) == len(act)
    kappa = np.zeros(max(n, 1), np.float64)
    out = np.zeros(max(n, 1), np.uint8)
    vp = _ViewPack(views, False)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    lib().oracle_surfel_coverage(_p(pts), _p(sc), _p(qs), n, _p(li), _p(origin), float(grid["voxel"]),
                                 int(grid["dim"]), _p(act), len(act), _p(vm), len(views),
                                 C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p), float(tau_M),
                                 float(tau_kappa), float(eps), _p(kappa), _p(out))
    return kappa[:n].copy(), out[:n].copy()


def surfel_view_counts(cam, mask, xyz, scale2, quat, tau_M=0.5, eps=1e-6):
    """(scored, total, mask_hit) of one surfel in one view (Pass 3 counts)."""
    c = _ocam(dict(cam, d_cam=0.0))
    m = np.ascontiguousarray(mask, np.float32)
    p = np.ascontiguousarray(xyz, np.float32)
    s2 = np.ascontiguousarray(scale2, np.float32)
    q = np.ascontiguousarray(quat, np.float32)
    tot, hit = C.c_int64(), C.c_int64()
    ok = lib().oracle_surfel_view_counts(C.byref(c), _p(m), float(tau_M), float(eps), _p(p), _p(s2), _p(q),
                                         C.byref(tot), C.byref(hit))
    return bool(ok), int(tot.value), int(hit.value)


def label(points, grid, seg_linear):
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    s = np.ascontiguousarray(seg_linear, dtype=np.uint32)
    out = np.zeros(max(len(pts), 1), np.uint8)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    lib().oracle_label(_p(pts), len(pts), _p(origin), float(grid["voxel"]), int(grid["dim"]), _p(s),
                       len(s), _p(out))
    return out[:len(pts)].copy()


def fuse_diff(active, grid, views, params):
    act = np.ascontiguousarray(active, dtype=np.uint32)
    n = len(act)
    P, W, Z = (np.zeros(max(n, 1)) for _ in range(3))
    vp = _ViewPack(views, False, use_logit=True)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    pr = _oparams(params)
    lib().oracle_fuse_diff(_p(act), n, _p(origin), float(grid["voxel"]), int(grid["dim"]), len(views),
                           C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p), C.byref(pr),
                           _p(P), _p(W), _p(Z))
    return P[:n].copy(), W[:n].copy(), Z[:n].copy()


def fuse_diff_grad(active, grid, views, params, grad_P):
    """Exact gradient of sum(grad_P * P) w.r.t. logits and the three depth maps of every view."""
    act = np.ascontiguousarray(active, dtype=np.uint32)
    gP = np.ascontiguousarray(grad_P, dtype=np.float64)
    n = len(act)
    vp = _ViewPack(views, False, use_logit=True)
    S = len(views)
    grads = {k: [np.zeros(v.dmed.shape, np.float64) for v in views] for k in ("logit", "dmin", "dmed", "dmax")}
    ptrs = {k: (C.c_void_p * max(S, 1))(*[_p(a).value for a in grads[k]]) for k in grads}
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    pr = _oparams(params)
    lib().oracle_fuse_diff_grad(_p(act), n, _p(origin), float(grid["voxel"]), int(grid["dim"]), S,
                                C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p), C.byref(pr),
                                _p(gP), C.cast(ptrs["logit"], C.c_void_p), C.cast(ptrs["dmin"], C.c_void_p),
                                C.cast(ptrs["dmed"], C.c_void_p), C.cast(ptrs["dmax"], C.c_void_p))
    return grads


def fuse_diff_branches(active, grid, views, params, coef):
    """Branches of the differentiable votes of the voxels with coef != 0:
    dict(votes, lo_clamp, hi_clamp, front, hw_floor, pixels_ge3, max_per_pixel)."""
    act = np.ascontiguousarray(active, dtype=np.uint32)
    cf = np.ascontiguousarray(coef, dtype=np.float64)
    out = np.zeros(7, np.int64)
    vp = _ViewPack(views, False, use_logit=True)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    pr = _oparams(params)
    lib().oracle_fuse_diff_branches(_p(act), len(act), _p(origin), float(grid["voxel"]), int(grid["dim"]),
                                    len(views), C.cast(vp.cams, C.c_void_p), C.cast(vp.maps, C.c_void_p),
                                    C.byref(pr), _p(cf), _p(out))
    keys = ("votes", "lo_clamp", "hi_clamp", "front", "hw_floor", "pixels_ge3", "max_per_pixel")
    return {k: int(v) for k, v in zip(keys, out)}


def pi_dg_map(dmin, dmax, k):
    dmin = np.ascontiguousarray(dmin, np.float32)
    dmax = np.ascontiguousarray(dmax, np.float32)
    H, W = dmin.shape
    out = np.zeros((H, W), np.float64)
    lib().oracle_pi_dg_map(_p(dmin), _p(dmax), W, H, float(k), _p(out))
    return out


def project(cam, p, eps=1e-6):
    c = _ocam(dict(cam, d_cam=0.0))
    pp = np.ascontiguousarray(p, np.float64)
    u, v, qz = C.c_double(), C.c_double(), C.c_double()
    ok = lib().oracle_project(C.byref(c), _p(pp), float(eps), C.byref(u), C.byref(v), C.byref(qz))
    return bool(ok), u.value, v.value, qz.value


def pixel_ray(cam, px, py):
    c = _ocam(dict(cam, d_cam=0.0))
    d = np.zeros(3)
    cs = C.c_double()
    lib().oracle_pixel_ray(C.byref(c), int(px), int(py), _p(d), C.byref(cs))
    return d, cs.value


def footprint_stats(nsamp, x0, x1, y0, y1, n):
    ns = np.ascontiguousarray(nsamp, np.uint16)
    lay, E = C.c_int(), C.c_double()
    lib().oracle_footprint_stats(_p(ns), ns.shape[1], x0, x1, y0, y1, int(n), C.byref(lay), C.byref(E))
    return bool(lay.value), E.value


def morton3(x, y, z):
    return int(lib().oracle_morton3(x, y, z))


def point_voxel(p, grid):
    pp = np.ascontiguousarray(p, np.float32)
    origin = np.ascontiguousarray(grid["origin"], np.float64)
    return int(lib().oracle_point_voxel(_p(pp), _p(origin), float(grid["voxel"]), int(grid["dim"])))


def num_threads():
    return int(lib().oracle_num_threads())


def reference_run(scene, params, use_nsamp=False, n_threads=1):
    """Occupancy -> fusion -> labels for a scene, timed (the CPU baseline)."""
    t0 = time.perf_counter()
    act = occupancy(scene.points, scene.grid)
    t1 = time.perf_counter()
    res = fuse(act, scene.grid, scene.views, params, use_nsamp=use_nsamp, n_threads=n_threads)
    t2 = time.perf_counter()
    seg_lin = act[res["seg"].astype(bool)]
    lab = label(scene.label_points, scene.grid, seg_lin)
    t3 = time.perf_counter()
    return dict(active=act, fuse=res, labels=lab, t_occ=t1 - t0, t_fuse=t2 - t1, t_label=t3 - t2)
