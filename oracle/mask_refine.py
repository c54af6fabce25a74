"""Depth refinement of a view's mask -- TEST INFRASTRUCTURE ONLY (oracle).

Plain numpy, binary64.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the HIP library never
does, and the two share no code.

It restates Sec. 3.2, "Depth-weighting", of DivAS (arXiv 2601.04860):

Band-pass (2DGS; Eq. depthband and Eq. gs-bandpass).  The median depth at each
positive prompt pixel and at the view centre forms the set D_s, whose minimum
and maximum bound the band; d_far is the 98th percentile of the median-depth
map.  Outside the band a pixel's weight falls off linearly to 0 at d_far:
    D_band = clip((max(d_min - D, 0) + max(D - d_max, 0))
                  / max(d_far - d_max, 1e-6), 0, 1),
    M~ = M (1 - D_band).

Min-max (NeRF; Eq. nerf-depthweight):
    M~ = M (1 - (D - min D) / (max D - min D)).

Readings where the paper is silent (each is listed in the design notes):
  - a pixel has a surface iff its depth is finite and > 0 (depth 0 means no
    surface in the library's map convention); d_far, min D and max D are taken
    over surface pixels only, and a pixel without a surface gets weight 0
    (it is treated as infinitely far);
  - the view centre is pixel (width // 2, height // 2); prompt and centre
    pixels without a surface do not enter D_s; with no anchor left the call
    is an error;
  - the percentile interpolates linearly between order statistics around
    position 0.98 (m - 1), as in the grid construction;
  - min-max with max D = min D gives every surface pixel weight 1;
  - the arithmetic is binary64 in the order written above, the mask value is
    widened from float32 and the product rounded once to float32.

Parity: bit-exact (exact order statistics and extrema, fixed operation order).
Pins: tests/test_oracle_refine_pins.py.
"""
from __future__ import annotations

import numpy as np

from .grid_stats import percentile_linear


def has_surface(d):
    d = np.asarray(d, dtype=np.float32)
    return np.isfinite(d) & (d > 0)


def depth_band(dmed, prompts_xy):
    """(d_min, d_max) of Eq. depthband: prompts_xy is a sequence of (x, y)."""
    dmed = np.asarray(dmed, dtype=np.float32)
    h, w = dmed.shape
    anchors = [(int(x), int(y)) for x, y in prompts_xy] + [(w // 2, h // 2)]
    vals = []
    for x, y in anchors:
        if not (0 <= x < w and 0 <= y < h):
            raise ValueError("prompt pixel outside the view")
        v = float(dmed[y, x])
        if np.isfinite(v) and v > 0:
            vals.append(v)
    if not vals:
        raise ValueError("no prompt or centre pixel has a surface")
    return min(vals), max(vals)


def far_depth(dmed, q=0.98):
    dmed = np.asarray(dmed, dtype=np.float32)
    vals = dmed[has_surface(dmed)].astype(np.float64)
    if vals.size == 0:
        raise ValueError("no pixel has a surface")
    return percentile_linear(vals, q)


def refine_bandpass(mask, dmed, prompts_xy):
    """Eq. gs-bandpass.  Returns (refined float32 plane, stats dict)."""
    mask = np.asarray(mask, dtype=np.float32)
    dmed = np.asarray(dmed, dtype=np.float32)
    lo, hi = depth_band(dmed, prompts_xy)
    d_far = far_depth(dmed)
    den = max(d_far - hi, 1e-6)
    D = dmed.astype(np.float64)
    dneg = np.maximum(lo - D, 0.0)
    dpos = np.maximum(D - hi, 0.0)
    band = np.minimum(np.maximum((dneg + dpos) / den, 0.0), 1.0)
    band = np.where(has_surface(dmed), band, 1.0)
    out = (mask.astype(np.float64) * (1.0 - band)).astype(np.float32)
    return out, dict(band_min=lo, band_max=hi, d_far=d_far, n_surface=int(has_surface(dmed).sum()))


def refine_minmax(mask, dexp):
    """Eq. nerf-depthweight.  Returns (refined float32 plane, stats dict)."""
    mask = np.asarray(mask, dtype=np.float32)
    dexp = np.asarray(dexp, dtype=np.float32)
    surf = has_surface(dexp)
    if not surf.any():
        raise ValueError("no pixel has a surface")
    D = dexp.astype(np.float64)
    zmin, zmax = float(D[surf].min()), float(D[surf].max())
    if zmax > zmin:
        z = (D - zmin) / (zmax - zmin)
    else:
        z = np.zeros_like(D)
    z = np.where(surf, z, 1.0)
    out = (mask.astype(np.float64) * (1.0 - z)).astype(np.float32)
    return out, dict(z_min=zmin, z_max=zmax, n_surface=int(surf.sum()))
