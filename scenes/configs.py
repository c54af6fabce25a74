"""Scene recipes for the workloads the library is measured and tested on.

  c1  tiny analytic: unit sphere on a ground square in [-1,1]^3, 64^3 grid,
      20k surface points, 4 pinhole views 128x96 at radius 3.
  c2  forward-facing: 20 random spheres/boxes, 300k points, 256^3 grid,
      10 views 504x378 on a jittered 5x2 grid looking along +z.
  c3  unbounded 360: 60 primitives inside a [-4,4]^3 box with a background
      shell, 3M points, 512^3 grid (~2% occupied), 16 views 1264x832 on a ring.
  c4  differentiable: the c1 scene with per-view soft-mask logits.
  grid scenes (serving): 360 scenes of 128^3..512^3 with several targets and
      click views made by the centroid-view camera update (move half-way to
      the clicked point, look at it).

The numbers of each recipe are documented in the design doc (input recipe).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy import ndimage

from .geometry import Box, InnerBox, Quad, Sphere, cast_rays, look_at_camera

CONFIG_NAMES = ("c1", "c2", "c3", "c4")


@dataclass
class View:
    cam: dict
    d_cam: float
    mask: np.ndarray           # float32 [H, W] in [0, 1] (soft mask of the target)
    dmin: np.ndarray           # float32 [H, W] planar depths, 0 = no surface
    dmed: np.ndarray
    dmax: np.ndarray
    nsamp: Optional[np.ndarray] = None   # uint16 [H, W] surface crossings
    logit: Optional[np.ndarray] = None   # float32 [H, W] (differentiable workload)
    masks: Optional[list] = None         # one float32 mask per target (grid scenes)
    prim_id: Optional[np.ndarray] = None
    # the same shell as distances along each pixel's ray (the depth semantics of
    # a NeRF renderer), float32 [H, W], 0 = no surface
    ray_dmin: Optional[np.ndarray] = None
    ray_dmed: Optional[np.ndarray] = None
    ray_dmax: Optional[np.ndarray] = None

    def as_ray_depth(self):
        """A copy whose depth planes are the ray-distance ones."""
        import copy
        v = copy.copy(self)
        v.dmin, v.dmed, v.dmax = self.ray_dmin, self.ray_dmed, self.ray_dmax
        return v


@dataclass
class Scene:
    name: str
    origin: np.ndarray         # float64 [3]
    voxel: float
    dim: int
    points: np.ndarray         # float32 [N, 3] occupancy points (Gaussian centres)
    views: List[View]
    prims: list = field(default_factory=list)
    target: int = 0
    targets: Optional[list] = None
    label_points: Optional[np.ndarray] = None
    info: dict = field(default_factory=dict)

    @property
    def grid(self):
        return dict(origin=np.asarray(self.origin, np.float64), voxel=float(self.voxel), dim=int(self.dim))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _soft_mask(inside, slope, noise_sd, rng, logit_noise_sd=None):
    """sigmoid(slope * signed pixel distance) + N(0, noise_sd), clipped to [0,1]."""
    if inside.any() and (~inside).any():
        d_in = ndimage.distance_transform_edt(inside)
        d_out = ndimage.distance_transform_edt(~inside)
        sd = np.where(inside, d_in - 0.5, -(d_out - 0.5))
    elif inside.any():
        sd = np.full(inside.shape, 1e3)
    else:
        sd = np.full(inside.shape, -1e3)
    z = slope * sd
    m = 1.0 / (1.0 + np.exp(-np.clip(z, -60, 60)))
    if noise_sd > 0:
        m = m + rng.normal(0.0, noise_sd, size=m.shape)
    m = np.clip(m, 0.0, 1.0).astype(np.float32)
    logit = None
    if logit_noise_sd is not None:
        logit = (z + rng.normal(0.0, logit_noise_sd, size=z.shape)).astype(np.float32)
    return m, logit


def _render_view(cam, prims, h, targets, rng, depth_noise=0.0, slope=8.0,
                 mask_noise=0.05, logit_noise=None, want_nsamp=True, d_cam=None, keep_pid=False):
    t, pid, cross, cos = cast_rays(cam, prims)
    hit = np.isfinite(t)
    tt = np.where(hit, t, 0.0)
    # shell model in ray space, converted to planar (camera-Z) depth
    rmin = np.where(hit, tt - 0.5 * h, 0.0)
    rmed = tt
    rmax = np.where(hit, tt + 0.5 * h, 0.0)
    tmin, tmed, tmax = rmin * cos, rmed * cos, rmax * cos
    if depth_noise > 0:
        f = 1.0 + depth_noise * rng.normal(size=t.shape)
        tmin, tmed, tmax = tmin * f, tmed * f, tmax * f
        rmin, rmed, rmax = rmin * f, rmed * f, rmax * f
    masks, logits = [], []
    for tg in targets:
        m, lg = _soft_mask(pid == tg, slope, mask_noise, rng, logit_noise)
        masks.append(m)
        logits.append(lg)
    ns = np.minimum(cross, 65535).astype(np.uint16) if want_nsamp else None
    return View(cam=cam, d_cam=float(d_cam), mask=masks[0], dmin=tmin.astype(np.float32),
                dmed=tmed.astype(np.float32), dmax=tmax.astype(np.float32), nsamp=ns,
                logit=logits[0], masks=masks, prim_id=pid if keep_pid else None,
                ray_dmin=rmin.astype(np.float32), ray_dmed=rmed.astype(np.float32),
                ray_dmax=rmax.astype(np.float32))


def _sample_surfaces(prims, n, rng, jitter_sd=0.0, weights=None):
    areas = np.array([p.area() for p in prims], dtype=np.float64)
    if weights is not None:
        areas = areas * np.asarray(weights, np.float64)
    counts = rng.multinomial(n, areas / areas.sum())
    pts = [p.sample(int(c), rng) for p, c in zip(prims, counts) if c > 0]
    pts = np.concatenate(pts, axis=0)
    if jitter_sd > 0:
        pts = pts + rng.normal(0.0, jitter_sd, size=pts.shape)
    pts = pts[rng.permutation(len(pts))]
    return pts.astype(np.float32)


def _ring_cams(n, radius, height, W, H, f, target=(0.0, 0.0, 0.0)):
    cams = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        pos = np.array([radius * math.cos(a), height, radius * math.sin(a)])
        cams.append(look_at_camera(pos, target, (0, 1, 0), f, f, W / 2.0, H / 2.0, W, H))
    return cams


# ---------------------------------------------------------------- c1 / c4
def make_tiny_sphere(seed=1, dim=64, n_points=20000, n_views=4, width=128, height=96,
                     focal=100.0, radius=3.0, elevation_deg=30.0, mask_noise=0.05,
                     logit_noise=None, depth_noise=0.0, slope=8.0):
    """Unit sphere (the target) resting on a ground square, in [-1,1]^3."""
    rng = _rng(seed)
    h = 2.0 / dim
    prims = [Sphere(np.zeros(3), 1.0), Quad(axis=1, value=-1.0, lo=(-1.0, -1.0), hi=(1.0, 1.0))]
    pts = _sample_surfaces(prims, n_points, rng)
    el = math.radians(elevation_deg)
    views = []
    for k in range(n_views):
        az = math.radians(45.0 + 360.0 * k / n_views)
        pos = radius * np.array([math.cos(el) * math.cos(az), math.sin(el), math.cos(el) * math.sin(az)])
        cam = look_at_camera(pos, (0, 0, 0), (0, 1, 0), focal, focal, width / 2.0, height / 2.0, width, height)
        views.append(_render_view(cam, prims, h, [0], rng, depth_noise=depth_noise, slope=slope,
                                  mask_noise=mask_noise, logit_noise=logit_noise, d_cam=radius))
    return Scene(name="c1", origin=np.array([-1.0, -1.0, -1.0]), voxel=h, dim=dim, points=pts,
                 views=views, prims=prims, target=0, label_points=pts)


def make_diff_scene(seed=4, **kw):
    """The c1 scene with per-view logits: 8 * signed pixel distance + N(0, 0.2)."""
    kw.setdefault("logit_noise", 0.2)
    s = make_tiny_sphere(seed=seed, **kw)
    s.name = "c4"
    return s


# ---------------------------------------------------------------- c2
def make_forward_facing(seed=2, dim=256, n_points=300_000, n_prims=20, n_views=10,
                        width=504, height=378, focal=400.0):
    rng = _rng(seed)
    prims = []
    for _ in range(n_prims):
        c = np.array([rng.uniform(-2, 2), rng.uniform(-1.5, 1.5), rng.uniform(3, 6)])
        if rng.random() < 0.5:
            prims.append(Sphere(c, float(rng.uniform(0.15, 0.5))))
        else:
            he = rng.uniform(0.15, 0.5, size=3)
            prims.append(Box(c - he, c + he))
    lo = np.min([p.bound()[0] - p.bound()[1] for p in prims], axis=0)
    hi = np.max([p.bound()[0] + p.bound()[1] for p in prims], axis=0)
    ctr = 0.5 * (lo + hi)
    half = 1.05 * 0.5 * float(np.max(hi - lo))
    origin = ctr - half
    h = 2.0 * half / dim
    pts = _sample_surfaces(prims, n_points, rng, jitter_sd=h / 4)
    scene_prims = prims + [Quad(axis=2, value=7.5, lo=(-6.0, -5.0), hi=(6.0, 5.0))]
    cams = []
    xs = np.linspace(-0.5, 0.5, 5)
    for j, y in enumerate((-0.25, 0.25)):
        for x in xs:
            pos = np.array([x + rng.uniform(-0.05, 0.05), y + rng.uniform(-0.05, 0.05), 0.0])
            cams.append(look_at_camera(pos, pos + np.array([0, 0, 1.0]), (0, 1, 0), focal, focal,
                                       width / 2.0, height / 2.0, width, height))
    cams = cams[:n_views]
    # target: the primitive with the most visible pixels in view 0
    _, pid0, _, _ = cast_rays(cams[0], scene_prims)
    vis = np.bincount(pid0[pid0 >= 0], minlength=len(scene_prims))[:n_prims]
    target = int(np.argmax(vis))
    tc = prims[target].bound()[0]
    views = [_render_view(c, scene_prims, h, [target], rng, depth_noise=0.01,
                          d_cam=float(np.linalg.norm(c["c2w"][:, 3] - tc))) for c in cams]
    return Scene(name="c2", origin=origin, voxel=h, dim=dim, points=pts, views=views,
                 prims=scene_prims, target=target, label_points=pts)


# ---------------------------------------------------------------- c3 / grid scenes
def _unbounded_prims(rng, n_prims, ball=2.0):
    prims = []
    for _ in range(n_prims):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        c = v * ball * rng.random() ** (1.0 / 3.0)
        if rng.random() < 0.5:
            prims.append(Sphere(c, float(rng.uniform(0.15, 0.5))))
        else:
            he = rng.uniform(0.15, 0.5, size=3)
            prims.append(Box(c - he, c + he))
    return prims


def make_unbounded(seed=3, dim=512, n_points=3_000_000, n_prims=60, n_views=16,
                   width=1264, height=832, focal=700.0, jitter_voxels=1.0, n_targets=1,
                   extent=4.0):
    """360 scene: primitives within radius 2, background shell at +-0.975*extent."""
    rng = _rng(seed)
    prims = _unbounded_prims(rng, n_prims)
    wall = 0.975 * extent
    shell = InnerBox(np.full(3, -wall), np.full(3, wall))
    all_prims = prims + [shell]
    h = 2.0 * extent / dim
    pts = _sample_surfaces(all_prims, n_points, rng, jitter_sd=jitter_voxels * h)
    dists = [float(np.linalg.norm(p.bound()[0])) for p in prims]
    order = list(np.argsort(dists))
    targets = [int(i) for i in order[:n_targets]]
    cams = _ring_cams(n_views, 3.0, 0.5, width, height, focal)
    views = []
    for c in cams:
        tc = prims[targets[0]].bound()[0]
        views.append(_render_view(c, all_prims, h, targets, rng,
                                  d_cam=float(np.linalg.norm(c["c2w"][:, 3] - tc))))
    return Scene(name="c3", origin=np.full(3, -extent), voxel=h, dim=dim, points=pts, views=views,
                 prims=all_prims, target=targets[0], targets=targets, label_points=pts)


def make_grid_scene(seed, dim, n_views, width, height, n_targets, n_points=None, n_prims=30,
                    focal=None):
    """A serving-workload scene: a 360 scene of grid ``dim`` with several targets."""
    if n_points is None:
        n_points = int(3_000_000 * (dim / 512) ** 2)
    if focal is None:
        focal = 0.55 * width
    s = make_unbounded(seed=seed, dim=dim, n_points=n_points, n_prims=n_prims, n_views=n_views,
                       width=width, height=height, focal=focal, n_targets=n_targets)
    s.name = f"grid{dim}"
    return s


def make_click_view(scene, rng, target_index=0, base_view=None, zoom=0.5, want_nsamp=False):
    """A click-driven centroid view: move the camera of a resident view half-way
    toward a point on the target and look at it; masks for every target."""
    if base_view is None:
        base_view = int(rng.integers(len(scene.views)))
    cam0 = scene.views[base_view].cam
    prim = scene.prims[scene.targets[target_index] if scene.targets else scene.target]
    c, r = prim.bound()
    x_t = c + rng.normal(0.0, 0.25 * r, size=3)
    p = cam0["c2w"][:, 3]
    p2 = p + zoom * (x_t - p)
    cam = look_at_camera(p2, x_t, (0, 1, 0), cam0["fx"], cam0["fy"], cam0["cx"], cam0["cy"],
                         cam0["width"], cam0["height"])
    targets = scene.targets if scene.targets else [scene.target]
    return _render_view(cam, scene.prims, scene.voxel, targets, rng, want_nsamp=want_nsamp,
                        d_cam=float(np.linalg.norm(p2 - x_t)))


SERVING_SCENES = ((128, 4, 504, 378, 1), (256, 8, 504, 378, 2), (512, 12, 1264, 832, 4), (512, 16, 1264, 832, 8))
SERVING_SCENES_SMALL = ((32, 3, 96, 72, 1), (64, 4, 128, 96, 2), (64, 5, 160, 120, 3))


def make_serving_workload(seed=5, small=False, pool=6):
    """Scenes of uneven size for the serving workload: (grid, resident views,
    view size, targets) per scene, a pool of click views per scene (centroid
    views toward one of its targets, masks for every target) and the
    (scene, target) pairs that sessions cycle over."""
    specs = SERVING_SCENES_SMALL if small else SERVING_SCENES
    rng = _rng(seed)
    out_scenes, pools = [], []
    for k, (dim, nv, W, H, nt) in enumerate(specs):
        npts = int(3_000_000 * (dim / 512) ** 2) if not small else int(4000 * (dim / 32) ** 2)
        s = make_unbounded(seed=seed * 100 + k, dim=dim, n_points=npts, n_prims=30, n_views=nv, width=W,
                           height=H, focal=0.55 * W, n_targets=nt)
        for v in s.views:
            v.nsamp = None
        s.name = f"serve{k}-{dim}"
        clicks = [make_click_view(s, rng, target_index=int(rng.integers(nt))) for _ in range(pool)]
        out_scenes.append(s)
        pools.append(clicks)
    pairs = [(k, t) for k, spec in enumerate(specs) for t in range(spec[4])]
    return dict(scenes=out_scenes, pools=pools, pairs=pairs, specs=specs)


def make_config(name, **kw):
    if name == "c1":
        return make_tiny_sphere(**kw)
    if name == "c2":
        return make_forward_facing(**kw)
    if name == "c3":
        return make_unbounded(**kw)
    if name == "c4":
        return make_diff_scene(**kw)
    raise ValueError(f"unknown config {name!r}")


_FORMAT = 2  # bumped when the pickled layout changes


def cached(name, builder, **kw):
    """Build a scene once per machine: pickled under $DIVAS_SCENE_CACHE
    (default /tmp/divas_scenes), keyed by the builder name and its arguments.
    The cache only holds files this module wrote itself."""
    import hashlib
    import os
    import pickle
    root = os.environ.get("DIVAS_SCENE_CACHE", "/tmp/divas_scenes")
    key = hashlib.sha1(repr((name, builder.__name__, sorted(kw.items()), _FORMAT)).encode()).hexdigest()[:16]
    path = os.path.join(root, f"{name}_{key}.pkl")
    if os.path.exists(path):
        try:
            with open(path, "rb") as f:
                return pickle.load(f)
        except Exception:
            pass
    scene = builder(**kw)
    try:
        os.makedirs(root, exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "wb") as f:
            pickle.dump(scene, f, protocol=pickle.HIGHEST_PROTOCOL)
        os.replace(tmp, path)
    except OSError:
        pass
    return scene


def config_scene(name, **kw):
    """The scene of a named workload, through the on-disk cache."""
    builders = {"c1": make_tiny_sphere, "c2": make_forward_facing, "c3": make_unbounded, "c4": make_diff_scene,
                "c5": make_serving_workload}
    return cached(name, builders[name], **kw)
