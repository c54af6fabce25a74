"""Analytic primitives, pinhole cameras and a ray caster for synthetic scenes.

Everything here is scene synthesis (the renderer and the surface sampler that
the paper's pipeline would get from a trained 2DGS / NeRF scene).  All
geometry is evaluated in float64; outputs are cast to float32 by the callers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_T_EPS = 1e-9


def _normalize(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def look_at_camera(pos, target, up, fx, fy, cx, cy, width, height):
    """OpenCV pinhole camera at ``pos`` looking at ``target``.

    Returns a dict with intrinsics, size and a 3x4 row-major ``c2w = [R | o]``
    whose columns are (right, down, forward, centre) in world coordinates.
    """
    pos = np.asarray(pos, dtype=np.float64)
    fwd = _normalize(np.asarray(target, dtype=np.float64) - pos)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    if np.linalg.norm(right) < 1e-12:  # looking along the up axis
        right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right = _normalize(right)
    down = np.cross(fwd, right)
    c2w = np.zeros((3, 4), dtype=np.float64)
    c2w[:, 0] = right
    c2w[:, 1] = down
    c2w[:, 2] = fwd
    c2w[:, 3] = pos
    return dict(fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy),
                c2w=c2w, width=int(width), height=int(height))


def pixel_rays(cam, xs=None, ys=None):
    """Unit world directions of the rays through pixel centres.

    With ``xs``/``ys`` (integer pixel coordinates, same shape) only those
    pixels are generated.  Returns (dirs[...,3], forward_cosine[...]).
    """
    W, H = cam["width"], cam["height"]
    if xs is None:
        ys, xs = np.mgrid[0:H, 0:W]
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    rc = np.stack([(xs + 0.5 - cam["cx"]) / cam["fx"],
                   (ys + 0.5 - cam["cy"]) / cam["fy"],
                   np.ones_like(xs)], axis=-1)
    R = cam["c2w"][:, :3]
    d = rc @ R.T
    n = np.linalg.norm(d, axis=-1, keepdims=True)
    d = d / n
    cos = d @ R[:, 2]
    return d, cos


@dataclass
class Sphere:
    center: np.ndarray
    radius: float

    def area(self):
        return 4.0 * math.pi * self.radius ** 2

    def bound(self):
        return np.asarray(self.center, np.float64), float(self.radius)

    def intersect(self, o, d):
        """First positive hit distance (inf if none) and number of crossings."""
        oc = o - np.asarray(self.center, np.float64)
        b = d @ oc if oc.ndim == 1 else np.einsum("ij,ij->i", d, oc)
        c = float(oc @ oc) - self.radius ** 2
        disc = b * b - c
        hit = disc >= 0.0
        s = np.sqrt(np.where(hit, disc, 0.0))
        t0 = -b - s
        t1 = -b + s
        first = np.where(t0 > _T_EPS, t0, np.where(t1 > _T_EPS, t1, np.inf))
        first = np.where(hit, first, np.inf)
        n = (hit & (t0 > _T_EPS)).astype(np.int32) + (hit & (t1 > _T_EPS)).astype(np.int32)
        return first, n

    def sample(self, n, rng):
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        return np.asarray(self.center, np.float64) + self.radius * v


def _slab(o, d, lo, hi):
    """Ray parameter interval inside the box [lo, hi] for rays o + t d (d: N x 3),
    one axis at a time."""
    o = np.broadcast_to(np.asarray(o, np.float64), d.shape)
    tmin = np.full(d.shape[0], -np.inf)
    tmax = np.full(d.shape[0], np.inf)
    for a in range(3):
        da = np.ascontiguousarray(d[:, a])
        oa = np.ascontiguousarray(o[:, a])
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / da
            t1 = (lo[a] - oa) * inv
            t2 = (hi[a] - oa) * inv
        lo_a = np.minimum(t1, t2)
        hi_a = np.maximum(t1, t2)
        # rays parallel to a slab: inside -> (-inf, inf), outside -> empty
        par = da == 0.0
        if par.any():
            inside = (oa >= lo[a]) & (oa <= hi[a])
            lo_a = np.where(par, np.where(inside, -np.inf, np.inf), lo_a)
            hi_a = np.where(par, np.where(inside, np.inf, -np.inf), hi_a)
        tmin = np.maximum(tmin, lo_a)
        tmax = np.minimum(tmax, hi_a)
    return tmin, tmax


@dataclass
class Box:
    """Axis-aligned solid box [lo, hi]; rays hit its outer faces."""
    lo: np.ndarray
    hi: np.ndarray

    def _faces(self):
        lo, hi = np.asarray(self.lo, np.float64), np.asarray(self.hi, np.float64)
        e = hi - lo
        out = []
        for ax in range(3):
            a1, a2 = [k for k in range(3) if k != ax]
            for side in (lo[ax], hi[ax]):
                out.append((ax, side, a1, a2, e[a1] * e[a2]))
        return out

    def area(self):
        return float(sum(f[4] for f in self._faces()))

    def bound(self):
        lo, hi = np.asarray(self.lo, np.float64), np.asarray(self.hi, np.float64)
        return 0.5 * (lo + hi), float(0.5 * np.linalg.norm(hi - lo))

    def intersect(self, o, d):
        tmin, tmax = _slab(o, d, np.asarray(self.lo, np.float64), np.asarray(self.hi, np.float64))
        hit = tmax >= np.maximum(tmin, 0.0)
        first = np.where(tmin > _T_EPS, tmin, np.where(tmax > _T_EPS, tmax, np.inf))
        first = np.where(hit, first, np.inf)
        n = (hit & (tmin > _T_EPS)).astype(np.int32) + (hit & (tmax > _T_EPS)).astype(np.int32)
        return first, n

    def sample(self, n, rng):
        faces = self._faces()
        areas = np.array([f[4] for f in faces])
        k = rng.choice(len(faces), size=n, p=areas / areas.sum())
        lo, hi = np.asarray(self.lo, np.float64), np.asarray(self.hi, np.float64)
        pts = lo + rng.random((n, 3)) * (hi - lo)
        for fi, (ax, side, _, _, _) in enumerate(faces):
            pts[k == fi, ax] = side
        return pts


@dataclass
class InnerBox(Box):
    """Background shell: the inner walls of [lo, hi], seen from inside."""

    def intersect(self, o, d):
        tmin, tmax = _slab(o, d, np.asarray(self.lo, np.float64), np.asarray(self.hi, np.float64))
        hit = (tmax >= np.maximum(tmin, 0.0)) & (tmax > _T_EPS)
        first = np.where(hit, tmax, np.inf)
        return first, hit.astype(np.int32)

    def bound(self):
        return None, None


@dataclass
class Quad:
    """Axis-aligned rectangle on the plane ``coord[axis] = value``."""
    axis: int
    value: float
    lo: tuple  # bounds of the two other axes, in increasing axis order
    hi: tuple

    def _axes(self):
        return [k for k in range(3) if k != self.axis]

    def area(self):
        return float((self.hi[0] - self.lo[0]) * (self.hi[1] - self.lo[1]))

    def bound(self):
        a1, a2 = self._axes()
        c = np.zeros(3)
        c[self.axis] = self.value
        c[a1] = 0.5 * (self.lo[0] + self.hi[0])
        c[a2] = 0.5 * (self.lo[1] + self.hi[1])
        r = 0.5 * math.hypot(self.hi[0] - self.lo[0], self.hi[1] - self.lo[1])
        return c, r

    def intersect(self, o, d):
        a1, a2 = self._axes()
        da = d[..., self.axis]
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (self.value - o[..., self.axis] if o.ndim > 1 else self.value - o[self.axis]) / da
        p1 = (o[..., a1] if o.ndim > 1 else o[a1]) + t * d[..., a1]
        p2 = (o[..., a2] if o.ndim > 1 else o[a2]) + t * d[..., a2]
        hit = (t > _T_EPS) & (p1 >= self.lo[0]) & (p1 <= self.hi[0]) & (p2 >= self.lo[1]) & (p2 <= self.hi[1])
        hit &= np.isfinite(t)
        first = np.where(hit, t, np.inf)
        return first, hit.astype(np.int32)

    def sample(self, n, rng):
        a1, a2 = self._axes()
        pts = np.zeros((n, 3))
        pts[:, self.axis] = self.value
        pts[:, a1] = self.lo[0] + rng.random(n) * (self.hi[0] - self.lo[0])
        pts[:, a2] = self.lo[1] + rng.random(n) * (self.hi[1] - self.lo[1])
        return pts


def _prim_pixel_box(cam, prim):
    """Conservative pixel rectangle covered by a primitive's bounding sphere."""
    c, r = prim.bound()
    if c is None:
        return None
    R = cam["c2w"][:, :3]
    o = cam["c2w"][:, 3]
    q = R.T @ (c - o)
    dist = float(np.linalg.norm(q))
    if dist <= r * 1.0001 or q[2] <= r:  # camera inside/behind the bound: no cull
        return None
    # angular radius of the bounding sphere, projected conservatively
    zmin = q[2] - r
    xs = [q[0] - r, q[0] + r]
    ys = [q[1] - r, q[1] + r]
    us = [cam["fx"] * x / zmin + cam["cx"] for x in xs] + [cam["fx"] * x / (q[2] + r) + cam["cx"] for x in xs]
    vs = [cam["fy"] * y / zmin + cam["cy"] for y in ys] + [cam["fy"] * y / (q[2] + r) + cam["cy"] for y in ys]
    x0 = max(int(math.floor(min(us))) - 2, 0)
    x1 = min(int(math.ceil(max(us))) + 2, cam["width"])
    y0 = max(int(math.floor(min(vs))) - 2, 0)
    y1 = min(int(math.ceil(max(vs))) + 2, cam["height"])
    return x0, x1, y0, y1


def cast_rays(cam, prims):
    """Ray-cast every pixel centre against ``prims``.

    Returns (t_hit[H,W] ray distance, inf on miss; prim_id[H,W], -1 on miss;
    crossings[H,W] surface crossings along the whole ray; cos[H,W]).
    """
    W, H = cam["width"], cam["height"]
    d, cos = pixel_rays(cam)
    o = cam["c2w"][:, 3].astype(np.float64)
    t_best = np.full((H, W), np.inf)
    pid = np.full((H, W), -1, dtype=np.int32)
    cross = np.zeros((H, W), dtype=np.int32)
    for k, prim in enumerate(prims):
        box = _prim_pixel_box(cam, prim)
        if box is None:
            sl = (slice(0, H), slice(0, W))
        else:
            x0, x1, y0, y1 = box
            if x0 >= x1 or y0 >= y1:
                continue
            sl = (slice(y0, y1), slice(x0, x1))
        dd = d[sl].reshape(-1, 3)
        t, n = prim.intersect(o, dd)
        t = t.reshape(t_best[sl].shape)
        n = n.reshape(t_best[sl].shape)
        better = t < t_best[sl]
        t_best[sl] = np.where(better, t, t_best[sl])
        pid[sl] = np.where(better, k, pid[sl])
        cross[sl] += n
    return t_best, pid, cross, cos
