"""Python binding of libdivas (depth-weighted voxel aggregation on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libdivas.so``.  PyTorch provides device memory and streams; the
ctypes structures below mirror ``include/divas.h``.  There is no fallback: if
the shared library is missing or fails to load, importing this package raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# PyTorch first: its HIP runtime is then the one the library binds to.  Loaded
# the other way round, the process would hold two HIP runtimes, and the
# second one to start finds no device.
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdivas.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdivas.so is not built at {LIB_PATH}; run __graft_entry__.build() "
                      "(or python paper_2601_04860_amd/build.py)")
_lib = C.CDLL(LIB_PATH)

OK, ERR_ARG, ERR_OOM, ERR_ADMISSION, ERR_TOO_MANY_VIEWS, ERR_STATE, ERR_DEVICE, ERR_CAPACITY = range(8)
MAX_VIEWS = 64

EXPORTS = ("divas_params_default", "divas_ctx_create", "divas_ctx_destroy", "divas_ctx_usage",
           "divas_session_footprint", "divas_session_create", "divas_session_rebuild", "divas_session_info",
           "divas_fuse_views", "divas_update_view", "divas_label_points", "divas_label_session_points",
           "divas_fuse_backward",
           "divas_session_destroy", "divas_status_string", "divas_last_error", "divas_session_set_timing",
           "divas_session_timings", "divas_batch_create", "divas_batch_run", "divas_batch_tune",
           "divas_batch_destroy", "divas_server_create", "divas_server_now", "divas_server_open_session",
           "divas_server_session", "divas_server_close_session", "divas_server_submit", "divas_server_wait",
           "divas_server_drain", "divas_server_stats", "divas_server_latencies", "divas_server_destroy",
           "divas_session_fusion_work", "divas_grid_params_default", "divas_grid_from_points",
           "divas_refine_mask_bandpass", "divas_refine_mask_minmax", "divas_params_nerf", "divas_needle_cull",
           "divas_needle_cull_noalloc", "divas_surfel_coverage", "divas_session_create_target",
           "divas_fuse_targets",
           "divas_session_generation", "divas_batch_validate")
BATCH_FUSE, BATCH_UPDATE = 0, 1
PHASES = ("occupancy", "views", "cull", "fuse", "label", "backward")


class Grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("voxel", C.c_double), ("dim", C.c_int32)]


class Occupancy(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("opacity", C.c_void_p), ("n", C.c_int64), ("tau_occ", C.c_double)]


class Camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("c2w", C.c_double * 12), ("width", C.c_int32), ("height", C.c_int32), ("d_cam", C.c_double)]


class ViewMaps(C.Structure):
    _fields_ = [("mask", C.c_void_p), ("d_min", C.c_void_p), ("d_ref", C.c_void_p), ("d_max", C.c_void_p),
                ("n_samp", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("gamma", "beta", "gamma_st", "alpha1", "k_grad", "eps", "tau_cons",
                                          "mask_gate", "soft_width")] + \
               [("differentiable", C.c_int32), ("retain_state", C.c_int32), ("variant", C.c_int32),
                ("lambda_range", C.c_double), ("b_max", C.c_double), ("thin", C.c_int32)] + \
               [(n, C.c_double) for n in ("rho_thin", "tau_thin", "rho_cover", "rho_occ", "n_abs")] + \
               [("nerf_ray_depths", C.c_int32), ("resident_outputs", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("P", C.c_void_p), ("vmask", C.c_void_p), ("seg_bits", C.c_void_p), ("counts", C.c_void_p)]


class BatchItem(C.Structure):
    _fields_ = [("session", C.c_void_p), ("op", C.c_int32), ("n_views", C.c_int32), ("slot", C.c_int32),
                ("pad", C.c_int32), ("cams", C.c_void_p), ("maps", C.c_void_p), ("out", Result)]


class BatchConfig(C.Structure):
    _fields_ = [("fuse_waves_per_block", C.c_int32), ("cull_blocks_per_cu", C.c_int32), ("use_graph", C.c_int32),
                ("schedule", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_batch", C.c_int32), ("max_new_views", C.c_int32),
                ("pad", C.c_int32), ("batch", BatchConfig)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("completed_updates", "batches", "batched_requests", "admission_waits",
                                         "max_queue", "failures", "sessions_open", "sessions_waiting")] + \
               [(n, C.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms")]


class GridParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("alpha_v", "beta_v", "pad", "percentile")] + \
               [("g0", C.c_int32), ("g_max", C.c_int32)]


class GridStats(C.Structure):
    _fields_ = [("center", C.c_double * 3)] + [(n, C.c_double) for n in ("r_fg", "b", "s_med", "h_v")] + \
               [("n_used", C.c_int64), ("n_kept", C.c_int64)]


class RefineStats(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("band_min", "band_max", "d_far", "z_min", "z_max")] + \
               [("n_surface", C.c_int64), ("n_anchors", C.c_int32)]


_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_sig = {
    "divas_params_default": ([C.c_double, _vp], C.c_int),
    "divas_params_nerf": ([C.c_double, _i32, _vp], C.c_int),
    "divas_needle_cull": ([_vp, _vp, _i64, C.c_double, _vp, _vp, _vp, _vp], C.c_int),
    "divas_needle_cull_noalloc": ([_vp, _vp, _i64, C.c_double, _vp, _vp, _vp, _vp], C.c_int),
    "divas_ctx_create": ([C.c_int, _sz, _vp], C.c_int),
    "divas_ctx_destroy": ([_vp], C.c_int),
    "divas_ctx_usage": ([_vp, _vp, _vp], C.c_int),
    "divas_session_footprint": ([_vp, _i64, _i32, _i64, _i32], _sz),
    "divas_session_create": ([_vp, _vp, _vp, _vp, _i64, _i32, _i64, _vp, _vp], C.c_int),
    "divas_session_rebuild": ([_vp, _vp, _vp], C.c_int),
    "divas_session_info": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "divas_fuse_views": ([_vp, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "divas_update_view": ([_vp, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "divas_label_points": ([_vp, _vp, _i64, _vp, _vp], C.c_int),
    "divas_label_session_points": ([_vp, _vp, _vp, _vp], C.c_int),
    "divas_session_create_target": ([_vp, _vp, _i32, _i64, _vp, _vp], C.c_int),
    "divas_fuse_targets": ([_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp], C.c_int),
    "divas_surfel_coverage": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp, C.c_double, C.c_double, _vp, _vp, _vp, _vp],
                              C.c_int),
    "divas_fuse_backward": ([_vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "divas_session_generation": ([_vp, _vp], C.c_int),
    "divas_batch_validate": ([_vp, _i32, _vp], C.c_int),
    "divas_session_destroy": ([_vp], C.c_int),
    "divas_status_string": ([C.c_int], C.c_char_p),
    "divas_session_set_timing": ([_vp, C.c_uint32], C.c_int),
    "divas_batch_create": ([_vp, _i32, _i32, _vp, _vp], C.c_int),
    "divas_batch_run": ([_vp, _i32, _vp, _vp], C.c_int),
    "divas_batch_tune": ([_vp, _i32, _vp, _vp, C.c_char_p, _vp], C.c_int),
    "divas_batch_destroy": ([_vp], C.c_int),
    "divas_server_create": ([_vp, _vp, _vp], C.c_int),
    "divas_server_now": ([_vp], C.c_double),
    "divas_server_open_session": ([_vp, _vp, _vp, _vp, _i64, _i32, _i64, _vp], C.c_int),
    "divas_server_session": ([_vp, _i32, _vp, _vp], C.c_int),
    "divas_server_close_session": ([_vp, _i32], C.c_int),
    "divas_server_submit": ([_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, C.c_double, _vp], C.c_int),
    "divas_server_wait": ([_vp, C.c_uint64, C.c_double, _vp, _vp], C.c_int),
    "divas_server_drain": ([_vp, C.c_double], C.c_int),
    "divas_server_stats": ([_vp, _vp], C.c_int),
    "divas_server_latencies": ([_vp, _vp, _i64, _vp], C.c_int),
    "divas_server_destroy": ([_vp], C.c_int),
    "divas_session_timings": ([_vp, _vp, _vp, _i32], C.c_int),
    "divas_last_error": ([], C.c_char_p),
    "divas_grid_params_default": ([_i32, _vp], C.c_int),
    "divas_grid_from_points": ([_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp], C.c_int),
    "divas_refine_mask_bandpass": ([_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp], C.c_int),
    "divas_refine_mask_minmax": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp], C.c_int),
}
for _name, (_args, _res) in _sig.items():
    if hasattr(_lib, _name):
        _f = getattr(_lib, _name)
        _f.argtypes = _args
        _f.restype = _res


class DivasError(RuntimeError):
    def __init__(self, status, where):
        self.status = int(status)
        msg = _lib.divas_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.divas_status_string(status).decode()} ({msg})")


def _check(st, where):
    if st != OK:
        raise DivasError(st, where)


def lib():
    return _lib


def default_params(voxel, **overrides):
    p = Params()
    _check(_lib.divas_params_default(float(voxel), C.byref(p)), "divas_params_default")
    for k, v in overrides.items():
        if v is None:
            continue
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, type(getattr(p, k))(v))
    return p


def nerf_params(voxel, column="360", **overrides):
    """Fusion constants of the NeRF thick path (Alg. nerf-fusion), column
    "llff" or "360" of the NeRF hyperparameter table."""
    p = Params()
    _check(_lib.divas_params_nerf(float(voxel), {"llff": 0, "360": 1}[column], C.byref(p)), "divas_params_nerf")
    for k, v in overrides.items():
        if v is None:
            continue
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, type(getattr(p, k))(v))
    return p


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t, dtype, name):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _vmask_ptr(t):
    torch = _torch()
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"vmask must be int64 or uint64, got {t.dtype}")
    return _dptr(t, t.dtype, "vmask")


def make_grid(origin, voxel, dim):
    g = Grid()
    for k in range(3):
        g.origin[k] = float(origin[k])
    g.voxel = float(voxel)
    g.dim = int(dim)
    return g


def make_camera(cam, d_cam):
    """cam: dict with fx, fy, cx, cy, c2w (3x4), width, height."""
    c = Camera()
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    flat = np.asarray(cam["c2w"], np.float64).reshape(12)
    for i in range(12):
        c.c2w[i] = float(flat[i])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.d_cam = float(d_cam)
    return c


def footprint(grid, max_points, max_views, max_view_pixels, retain_state=False):
    g = grid if isinstance(grid, Grid) else make_grid(**grid)
    return int(_lib.divas_session_footprint(C.byref(g), int(max_points), int(max_views), int(max_view_pixels),
                                            int(bool(retain_state))))


def grid_from_points(ctx, xyz, scale=None, g_max=512, stream=None, **overrides):
    """Scene-statistic grid (Eq. scene-norm, Eq. voxel-size) of device points.

    xyz: float32 CUDA tensor [n, 3]; scale: float32 CUDA tensor [n] or None.
    Returns (grid dict usable by Session, stats dict)."""
    torch = _torch()
    p = GridParams()
    _check(_lib.divas_grid_params_default(int(g_max), C.byref(p)), "divas_grid_params_default")
    for k, v in overrides.items():
        setattr(p, k, v)
    n = int(xyz.shape[0]) if xyz.dim() == 2 else int(xyz.numel() // 3)
    g, st = Grid(), GridStats()
    _check(_lib.divas_grid_from_points(ctx.handle, _dptr(xyz, torch.float32, "xyz"),
                                       _dptr(scale, torch.float32, "scale"), n, C.byref(p), C.byref(g),
                                       C.byref(st), _stream(stream)), "divas_grid_from_points")
    grid = dict(origin=[g.origin[k] for k in range(3)], voxel=g.voxel, dim=g.dim)
    stats = dict(center=[st.center[k] for k in range(3)], r_fg=st.r_fg, b=st.b, s_med=st.s_med, h_v=st.h_v,
                 n_used=st.n_used, n_kept=st.n_kept)
    return grid, stats


def _needle(fn, ctx, scales, labels, eps, stream):
    torch = _torch()
    n = int(labels.numel())
    if int(scales.numel()) != 2 * n:
        raise ValueError("scales must hold two values per label")
    tau, cut = C.c_double(), C.c_int64()
    _check(getattr(_lib, fn)(ctx.handle, _dptr(scales, torch.float32, "scales"), n, float(eps),
                             _dptr(labels, torch.uint8, "labels"), C.byref(tau), C.byref(cut), _stream(stream)), fn)
    return tau.value, cut.value


def needle_cull(ctx, scales, labels, eps=1e-6, stream=None):
    """Pass 2 of the voxel-to-surfel mapping (Eq. aspect, Eq. needle,
    Eq. pass-needle) on device tensors: scales float32 [n, 2], labels uint8 [n]
    (updated in place).  Returns (tau_a, n_culled)."""
    return _needle("divas_needle_cull", ctx, scales, labels, eps, stream)


NOALLOC_MAX_SURFELS = 4000000


def needle_cull_noalloc(ctx, scales, labels, eps=1e-6, stream=None):
    """needle_cull on the library's fixed device scratch: no device
    allocation, at most NOALLOC_MAX_SURFELS surfels.  Calls that overlap on
    one device race."""
    return _needle("divas_needle_cull_noalloc", ctx, scales, labels, eps, stream)


TARGET_SCHEDULES = {"auto": 0, "together": 1, "one_by_one": 2}


def fuse_targets(sessions, viewsets, results, stream=None, schedule="auto"):
    """divas_fuse_targets: sessions of one scene (a session and target sessions
    of it), viewsets[t] target t's views (ViewSet.with_masks of one depth set),
    results[t] its result dict (Session.alloc_result); schedule "auto",
    "together" or "one_by_one"."""
    if schedule not in TARGET_SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(TARGET_SCHEDULES)}")
    T = len(sessions)
    if len(viewsets) != T or len(results) != T:
        raise ValueError("one view set and one result per session")
    n = len(viewsets[0].cams) if T else 0
    if any(len(v.cams) != n for v in viewsets):
        raise ValueError("every target needs the same number of views")
    hs = (C.c_void_p * max(T, 1))(*[s.handle for s in sessions])
    cams = (Camera * max(n, 1))(*viewsets[0].cams)
    maps = (ViewMaps * max(T * n, 1))(*[m for v in viewsets for m in v.maps])
    outs = (Result * max(T, 1))(*[Session._result(r) for r in results])
    _check(_lib.divas_fuse_targets(C.cast(hs, C.c_void_p), T, n, C.cast(cams, C.c_void_p), C.cast(maps, C.c_void_p),
                                   C.cast(outs, C.c_void_p), TARGET_SCHEDULES[schedule], _stream(stream)),
           "divas_fuse_targets")
    return results


def _refine_stats(st):
    return dict(band_min=st.band_min, band_max=st.band_max, d_far=st.d_far, z_min=st.z_min, z_max=st.z_max,
                n_surface=st.n_surface, n_anchors=st.n_anchors)


def refine_mask_bandpass(ctx, mask, d_med, prompts_xy=(), out=None, stream=None):
    """Band-pass depth refinement (Eq. depthband, Eq. gs-bandpass) of one view.

    mask, d_med: float32 CUDA tensors [H, W]; prompts_xy: (x, y) pixel pairs.
    Returns (refined tensor, stats dict)."""
    torch = _torch()
    h, w = int(mask.shape[0]), int(mask.shape[1])
    out = torch.empty_like(mask) if out is None else out
    pr = np.ascontiguousarray(np.asarray(prompts_xy, np.int32).reshape(-1, 2))
    st = RefineStats()
    _check(_lib.divas_refine_mask_bandpass(ctx.handle, w, h, _dptr(mask, torch.float32, "mask"),
                                           _dptr(d_med, torch.float32, "d_med"),
                                           pr.ctypes.data if len(pr) else None, len(pr),
                                           _dptr(out, torch.float32, "out"), C.byref(st), _stream(stream)),
           "divas_refine_mask_bandpass")
    return out, _refine_stats(st)


def refine_mask_minmax(ctx, mask, d_exp, out=None, stream=None):
    """Min-max depth refinement (Eq. nerf-depthweight) of one view."""
    torch = _torch()
    h, w = int(mask.shape[0]), int(mask.shape[1])
    out = torch.empty_like(mask) if out is None else out
    st = RefineStats()
    _check(_lib.divas_refine_mask_minmax(ctx.handle, w, h, _dptr(mask, torch.float32, "mask"),
                                         _dptr(d_exp, torch.float32, "d_exp"), _dptr(out, torch.float32, "out"),
                                         C.byref(st), _stream(stream)), "divas_refine_mask_minmax")
    return out, _refine_stats(st)


class Context:
    def __init__(self, device=0, hbm_budget_bytes=0):
        self._h = C.c_void_p()
        _check(_lib.divas_ctx_create(int(device), int(hbm_budget_bytes), C.byref(self._h)), "divas_ctx_create")
        self.device = device

    @property
    def handle(self):
        return self._h

    def usage(self):
        u, b = C.c_size_t(), C.c_size_t()
        _check(_lib.divas_ctx_usage(self._h, C.byref(u), C.byref(b)), "divas_ctx_usage")
        return u.value, b.value

    def close(self):
        if self._h:
            _check(_lib.divas_ctx_destroy(self._h), "divas_ctx_destroy")
            self._h = C.c_void_p()


class ViewSet:
    """Cameras and device maps of several views, kept alive together."""

    def __init__(self):
        self.cams = []
        self.maps = []
        self.keep = []

    def add(self, cam, d_cam, mask, d_min, d_ref, d_max, n_samp=None):
        torch = _torch()
        m = ViewMaps(_dptr(mask, torch.float32, "mask"), _dptr(d_min, torch.float32, "d_min"),
                     _dptr(d_ref, torch.float32, "d_ref"), _dptr(d_max, torch.float32, "d_max"),
                     _dptr(n_samp, torch.int16, "n_samp") if n_samp is not None and n_samp.dtype == torch.int16
                     else _dptr(n_samp, torch.uint16, "n_samp") if n_samp is not None else None)
        self.cams.append(make_camera(cam, d_cam))
        self.maps.append(m)
        self.keep.append((mask, d_min, d_ref, d_max, n_samp))
        return len(self.cams) - 1

    def with_masks(self, masks):
        """The same views (cameras, depth planes, n_samp) with other mask
        planes: masks[k] (device float32 tensor) replaces view k's mask."""
        torch = _torch()
        if len(masks) != len(self.cams):
            raise ValueError("one mask per view")
        vs = ViewSet()
        vs.cams = list(self.cams)
        for m0, keep, mk in zip(self.maps, self.keep, masks):
            vs.maps.append(ViewMaps(_dptr(mk, torch.float32, "mask"), m0.d_min, m0.d_ref, m0.d_max, m0.n_samp))
            vs.keep.append((mk,) + tuple(keep[1:]))
        return vs

    def subset(self, b=0, e=None):
        """Views [b, e) as a ViewSet of their own (same device maps)."""
        e = len(self.cams) if e is None else e
        vs = ViewSet()
        vs.cams, vs.maps, vs.keep = self.cams[b:e], self.maps[b:e], self.keep[b:e]
        return vs

    def arrays(self, b=0, e=None):
        e = len(self.cams) if e is None else e
        n = e - b
        cams = (Camera * max(n, 1))(*self.cams[b:e])
        maps = (ViewMaps * max(n, 1))(*self.maps[b:e])
        return n, cams, maps


class Session:
    """A resident voxel grid: active list, accumulators, segmentation bitfield."""

    def __init__(self, ctx, grid, xyz, opacity=None, tau_occ=0.5, params=None, max_views=16,
                 max_view_pixels=1264 * 832, stream=None, max_points=0):
        torch = _torch()
        self.ctx = ctx
        self.grid = grid if isinstance(grid, Grid) else make_grid(**grid)
        self.params = params if params is not None else default_params(self.grid.voxel)
        n = int(xyz.shape[0])
        occ = Occupancy(_dptr(xyz, torch.float32, "xyz") if n else None,
                        _dptr(opacity, torch.float32, "opacity"), n, float(tau_occ))
        self._xyz = (xyz, opacity)
        self._h = C.c_void_p()
        _check(_lib.divas_session_create(self.ctx.handle, C.byref(self.grid), C.byref(occ), C.byref(self.params),
                                         int(max_points), int(max_views), int(max_view_pixels), _stream(stream),
                                         C.byref(self._h)), "divas_session_create")
        self.max_views = int(max_views)

    @classmethod
    def target(cls, base, params=None, max_views=16, max_view_pixels=1264 * 832, stream=None):
        """A target session over base's scene (shared occupancy; own views,
        parameters and results)."""
        self = cls.__new__(cls)
        self.ctx = base.ctx
        self.grid = base.grid
        self.params = params if params is not None else default_params(self.grid.voxel)
        self._xyz = None
        self._base = base  # kept alive while the target lives
        self._h = C.c_void_p()
        _check(_lib.divas_session_create_target(base.handle, C.byref(self.params), int(max_views),
                                                int(max_view_pixels), _stream(stream), C.byref(self._h)),
               "divas_session_create_target")
        self.max_views = int(max_views)
        return self

    @property
    def handle(self):
        return self._h

    def rebuild(self, xyz, opacity=None, tau_occ=0.5, stream=None):
        torch = _torch()
        occ = Occupancy(_dptr(xyz, torch.float32, "xyz") if xyz.shape[0] else None,
                        _dptr(opacity, torch.float32, "opacity"), int(xyz.shape[0]), float(tau_occ))
        self._xyz = xyz
        _check(_lib.divas_session_rebuild(self._h, C.byref(occ), _stream(stream)), "divas_session_rebuild")

    def info(self):
        n, act, nv, fp = C.c_int64(), C.c_void_p(), C.c_int32(), C.c_size_t()
        _check(_lib.divas_session_info(self._h, C.byref(n), C.byref(act), C.byref(nv), C.byref(fp)),
               "divas_session_info")
        return dict(n_active=n.value, active_ptr=act.value, n_views=nv.value, footprint=fp.value)

    def active_indices(self):
        """Copy of the Morton-ordered active list (linear voxel indices) as int64 numpy."""
        torch = _torch()
        inf = self.info()
        n = inf["n_active"]
        if n == 0:
            return np.zeros(0, np.int64)
        view = torch.as_tensor(_DeviceArray(inf["active_ptr"], n, "<i4"), device=f"cuda:{self.ctx.device}")
        return view.cpu().numpy().view(np.uint32).astype(np.int64)

    def alloc_result(self, with_bits=False):
        torch = _torch()
        n = max(self.info()["n_active"], 1)
        dev = f"cuda:{self.ctx.device}"
        P = torch.empty(n, dtype=torch.float32, device=dev)
        v = torch.empty(n, dtype=torch.int64, device=dev)
        counts = torch.zeros(3, dtype=torch.int64, device=dev)
        nw = max((self.grid.dim ** 3 + 31) // 32, 1)
        bits = torch.empty(nw, dtype=torch.int32, device=dev) if with_bits else None
        return dict(P=P, vmask=v, counts=counts, seg_bits=bits)

    @staticmethod
    def _result(res):
        return Result(res["P"].data_ptr(), res["vmask"].data_ptr(),
                      res["seg_bits"].data_ptr() if res.get("seg_bits") is not None else None,
                      res["counts"].data_ptr() if res.get("counts") is not None else None)

    def fuse_views(self, views: ViewSet, res=None, stream=None):
        res = res if res is not None else self.alloc_result()
        n, cams, maps = views.arrays()
        r = self._result(res)
        _check(_lib.divas_fuse_views(self._h, n, C.cast(cams, C.c_void_p), C.cast(maps, C.c_void_p), C.byref(r),
                                     _stream(stream)), "divas_fuse_views")
        self._views = views
        return res

    def update_view(self, slot, views: ViewSet, index, res=None, stream=None):
        res = res if res is not None else self.alloc_result()
        r = self._result(res)
        _check(_lib.divas_update_view(self._h, int(slot), C.byref(views.cams[index]), C.byref(views.maps[index]),
                                      C.byref(r), _stream(stream)), "divas_update_view")
        return res

    def label_points(self, xyz, labels=None, stream=None):
        torch = _torch()
        n = int(xyz.shape[0])
        if labels is None:
            labels = torch.empty(max(n, 1), dtype=torch.uint8, device=xyz.device)
        if labels.numel() < n:
            raise ValueError(f"labels holds {labels.numel()} entries, {n} needed")
        _check(_lib.divas_label_points(self._h, _dptr(xyz, torch.float32, "xyz") if n else None, n,
                                       _dptr(labels, torch.uint8, "labels"), _stream(stream)), "divas_label_points")
        return labels[:n]

    def label_session_points(self, labels=None, stream=None):
        """Labels of the points of the session's last occupancy build (for a
        target session, its base's), from the voxel codes that build kept: the
        values label_points gives for those points."""
        torch = _torch()
        n = C.c_int64(0)
        _check(_lib.divas_label_session_points(self._h, None, C.byref(n), None), "divas_label_session_points")
        if labels is None:
            labels = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
        if labels.numel() < n.value:
            raise ValueError(f"labels holds {labels.numel()} entries, {n.value} needed")
        _check(_lib.divas_label_session_points(self._h, _dptr(labels, torch.uint8, "labels"), C.byref(n),
                                               _stream(stream)), "divas_label_session_points")
        return labels[:n.value]

    def surfel_coverage(self, xyz, scales, quats, labels_in, vmask, tau_M=0.5, tau_kappa=0.5, labels_out=None,
                        stream=None):
        """Pass 3 of the voxel-to-surfel mapping (Alg. vox2surfel; Eqs.
        cov-atomics, kappa, final-F) on device tensors: xyz float32 [n, 3],
        scales float32 [n, 2], quats float32 [n, 4] (w, x, y, z), labels_in
        uint8 [n], vmask int64/uint64 [n_active] (the last fusion's view
        bitmasks).  Returns (kappa float64 [n], labels uint8 [n], kept int64
        [1]) on the device."""
        torch = _torch()
        n = int(xyz.shape[0])
        for t, k, name in ((scales, 2, "scales"), (quats, 4, "quats"), (labels_in, 1, "labels_in")):
            if int(t.numel()) != k * n:
                raise ValueError(f"{name} must hold {k} values per surfel")
        dev = xyz.device
        kappa = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        if labels_out is None:
            labels_out = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        kept = torch.empty(1, dtype=torch.int64, device=dev)
        ptr = (lambda t, dt, nm: _dptr(t, dt, nm) if n else None)
        _check(_lib.divas_surfel_coverage(self._h, ptr(xyz, torch.float32, "xyz"), ptr(scales, torch.float32, "scales"),
                                          ptr(quats, torch.float32, "quats"), n,
                                          ptr(labels_in, torch.uint8, "labels_in"), _vmask_ptr(vmask),
                                          float(tau_M), float(tau_kappa), ptr(kappa, torch.float64, "kappa"),
                                          ptr(labels_out, torch.uint8, "labels_out"),
                                          _dptr(kept, torch.int64, "kept"), _stream(stream)),
               "divas_surfel_coverage")
        return kappa[:n], labels_out[:n], kept

    def fuse_backward(self, grad_P, grads, stream=None):
        """grads: dict key -> list (per view) of float32 HxW tensors or None; keys
        logit, dmin, dref, dmax."""
        torch = _torch()
        arrs = []
        n_views = self.info()["n_views"]
        for k in ("logit", "dmin", "dref", "dmax"):
            lst = grads.get(k)
            if lst is None:
                arrs.append(None)
                continue
            if len(lst) != n_views:
                raise ValueError(f"{k}: {len(lst)} gradient maps for {n_views} fused views")
            ptrs = (C.c_void_p * max(len(lst), 1))(*[None if t is None else _dptr(t, torch.float32, k) for t in lst])
            arrs.append(ptrs)
        self._bw_keep = arrs
        _check(_lib.divas_fuse_backward(self._h, _dptr(grad_P, torch.float32, "grad_P"), n_views,
                                        *[None if a is None else C.cast(a, C.c_void_p) for a in arrs],
                                        _stream(stream)), "divas_fuse_backward")

    def generation(self):
        """Counter bumped by every call that changes the fused state."""
        g = C.c_uint64()
        _check(_lib.divas_session_generation(self._h, C.byref(g)), "divas_session_generation")
        return g.value

    def fusion_work(self):
        """Hot chunks, hot (chunk, view) pairs and gathered samples of the last fusion."""
        v = [C.c_int64() for _ in range(3)]
        _check(_lib.divas_session_fusion_work(self._h, *[C.byref(x) for x in v]), "divas_session_fusion_work")
        return dict(hot_chunks=v[0].value, hot_pairs=v[1].value, gathered=v[2].value)

    def set_timing(self, enable=True, phases=None):
        """Time every phase (enable), none, or the named phases only."""
        mask = 0
        if phases is not None:
            for p in phases:
                mask |= 1 << PHASES.index(p)
        elif enable:
            mask = 0xFFFFFFFF
        _check(_lib.divas_session_set_timing(self._h, mask), "divas_session_set_timing")

    def timings(self, reset=False):
        """{phase: (milliseconds, launches)} accumulated since the last reset."""
        ms = (C.c_double * len(PHASES))()
        n = (C.c_int64 * len(PHASES))()
        _check(_lib.divas_session_timings(self._h, ms, n, int(bool(reset))), "divas_session_timings")
        return {p: (ms[i], n[i]) for i, p in enumerate(PHASES)}

    def close(self):
        if self._h:
            _check(_lib.divas_session_destroy(self._h), "divas_session_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many sessions in one persistent launch sequence (optionally a HIP graph)."""

    def __init__(self, ctx, max_items, max_new_views, fuse_waves_per_block=0, cull_blocks_per_cu=0, use_graph=True,
                 schedule=0):
        self.ctx = ctx
        cfg = BatchConfig(int(fuse_waves_per_block), int(cull_blocks_per_cu), int(bool(use_graph)), int(schedule))
        self._h = C.c_void_p()
        _check(_lib.divas_batch_create(ctx.handle, int(max_items), int(max_new_views), C.byref(cfg),
                                       C.byref(self._h)), "divas_batch_create")
        self._keep = None

    def _items(self, work):
        """work: list of (session, op, views: ViewSet, view index or None, slot, result dict)."""
        arr = (BatchItem * max(len(work), 1))()
        keep = []
        for k, (sess, op, vs, index, slot, res) in enumerate(work):
            if op == BATCH_FUSE:
                n, cams, maps = vs.arrays()
            else:
                n = 1
                cams = (Camera * 1)(vs.cams[index])
                maps = (ViewMaps * 1)(vs.maps[index])
            keep += [cams, maps]
            arr[k] = BatchItem(sess.handle.value, int(op), int(n), int(slot), 0, C.cast(cams, C.c_void_p),
                               C.cast(maps, C.c_void_p), Session._result(res))
        return arr, keep

    def run(self, work, stream=None):
        arr, keep = self._items(work)
        self._keep = (arr, keep, work)
        _check(_lib.divas_batch_run(self._h, len(work), arr, _stream(stream)), "divas_batch_run")

    def tune(self, work, cache_path=None, stream=None):
        arr, keep = self._items(work)
        self._keep = (arr, keep, work)
        cfg = BatchConfig()
        _check(_lib.divas_batch_tune(self._h, len(work), arr, _stream(stream),
                                     None if cache_path is None else str(cache_path).encode(), C.byref(cfg)),
               "divas_batch_tune")
        return dict(fuse_waves_per_block=cfg.fuse_waves_per_block, cull_blocks_per_cu=cfg.cull_blocks_per_cu,
                    use_graph=cfg.use_graph, schedule=cfg.schedule)

    def close(self):
        if self._h:
            _check(_lib.divas_batch_destroy(self._h), "divas_batch_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (native scheduler thread in libdivas)."""

    def __init__(self, ctx, n_streams=2, max_batch=64, max_new_views=64, use_graph=True, fuse_waves_per_block=0,
                 cull_blocks_per_cu=0):
        self.ctx = ctx
        cfg = ServerConfig(int(n_streams), int(max_batch), int(max_new_views), 0,
                           BatchConfig(int(fuse_waves_per_block), int(cull_blocks_per_cu), int(bool(use_graph)), 0))
        self._h = C.c_void_p()
        _check(_lib.divas_server_create(ctx.handle, C.byref(cfg), C.byref(self._h)), "divas_server_create")
        self._keep = {}      # ticket -> objects that must outlive the request
        self._sess_keep = {}  # sid -> (grid, occ, params, xyz)

    def now(self):
        return float(_lib.divas_server_now(self._h))

    def open_session(self, grid, xyz, params, opacity=None, tau_occ=0.5, max_points=0, max_views=16,
                     max_view_pixels=1264 * 832):
        torch = _torch()
        g = grid if isinstance(grid, Grid) else make_grid(**grid)
        n = int(xyz.shape[0])
        occ = Occupancy(_dptr(xyz, torch.float32, "xyz") if n else None, _dptr(opacity, torch.float32, "opacity"),
                        n, float(tau_occ))
        sid = C.c_int32()
        _check(_lib.divas_server_open_session(self._h, C.byref(g), C.byref(occ), C.byref(params), int(max_points),
                                              int(max_views), int(max_view_pixels), C.byref(sid)),
               "divas_server_open_session")
        self._sess_keep[sid.value] = (g, occ, params, xyz, opacity)
        return sid.value

    def session(self, sid):
        h, adm = C.c_void_p(), C.c_int32()
        _check(_lib.divas_server_session(self._h, int(sid), C.byref(h), C.byref(adm)), "divas_server_session")
        return h.value, adm.value

    def close_session(self, sid):
        _check(_lib.divas_server_close_session(self._h, int(sid)), "divas_server_close_session")

    def submit(self, sid, op, views, index, slot, res, arrival=-1.0):
        if op == BATCH_FUSE:
            n, cams, maps = views.arrays()
        else:
            n = 1
            cams = (Camera * 1)(views.cams[index])
            maps = (ViewMaps * 1)(views.maps[index])
        r = Session._result(res)
        t = C.c_uint64()
        _check(_lib.divas_server_submit(self._h, int(sid), int(op), int(n), int(slot), C.cast(cams, C.c_void_p),
                                        C.cast(maps, C.c_void_p), C.byref(r), float(arrival), C.byref(t)),
               "divas_server_submit")
        self._keep[t.value] = (views, res)
        return t.value

    def wait(self, ticket, timeout=10.0):
        done, lat = C.c_int32(), C.c_double()
        _check(_lib.divas_server_wait(self._h, C.c_uint64(ticket), float(timeout), C.byref(done), C.byref(lat)),
               "divas_server_wait")
        if done.value:
            self._keep.pop(ticket, None)
        return bool(done.value), lat.value

    def drain(self, timeout=60.0):
        _check(_lib.divas_server_drain(self._h, float(timeout)), "divas_server_drain")

    def stats(self):
        st = ServerStats()
        _check(_lib.divas_server_stats(self._h, C.byref(st)), "divas_server_stats")
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def latencies(self):
        n = C.c_int64()
        _check(_lib.divas_server_latencies(self._h, None, 0, C.byref(n)), "divas_server_latencies")
        arr = (C.c_double * max(n.value, 1))()
        _check(_lib.divas_server_latencies(self._h, arr, n.value, C.byref(n)), "divas_server_latencies")
        return np.array(arr[:n.value])

    def close(self):
        if self._h:
            _check(_lib.divas_server_destroy(self._h), "divas_server_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def session_info(handle):
    """n_active of a session handle (e.g. one owned by a Server)."""
    n = C.c_int64()
    _check(_lib.divas_session_info(C.c_void_p(handle), C.byref(n), None, None, None), "divas_session_info")
    return n.value


class _DeviceArray:
    """Zero-copy view of a library-owned device array (``__cuda_array_interface__``)."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 3, "strides": None}
