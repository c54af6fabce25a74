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
           "divas_fuse_views", "divas_update_view", "divas_label_points", "divas_fuse_backward",
           "divas_session_destroy", "divas_status_string", "divas_last_error")


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
               [("differentiable", C.c_int32), ("retain_state", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("P", C.c_void_p), ("vmask", C.c_void_p), ("seg_bits", C.c_void_p), ("counts", C.c_void_p)]


_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_sig = {
    "divas_params_default": ([C.c_double, _vp], C.c_int),
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
    "divas_fuse_backward": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "divas_session_destroy": ([_vp], C.c_int),
    "divas_status_string": ([C.c_int], C.c_char_p),
    "divas_last_error": ([], C.c_char_p),
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
        _check(_lib.divas_label_points(self._h, _dptr(xyz, torch.float32, "xyz") if n else None, n,
                                       labels.data_ptr(), _stream(stream)), "divas_label_points")
        return labels[:n]

    def fuse_backward(self, grad_P, grads, stream=None):
        """grads: dict key -> list (per view) of float32 HxW tensors or None; keys
        logit, dmin, dref, dmax."""
        torch = _torch()
        arrs = []
        for k in ("logit", "dmin", "dref", "dmax"):
            lst = grads.get(k)
            if lst is None:
                arrs.append(None)
                continue
            ptrs = (C.c_void_p * max(len(lst), 1))(*[None if t is None else _dptr(t, torch.float32, k) for t in lst])
            arrs.append(ptrs)
        self._bw_keep = arrs
        _check(_lib.divas_fuse_backward(self._h, _dptr(grad_P, torch.float32, "grad_P"),
                                        *[None if a is None else C.cast(a, C.c_void_p) for a in arrs],
                                        _stream(stream)), "divas_fuse_backward")

    def close(self):
        if self._h:
            _check(_lib.divas_session_destroy(self._h), "divas_session_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Zero-copy view of a library-owned device array (``__cuda_array_interface__``)."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 3, "strides": None}
