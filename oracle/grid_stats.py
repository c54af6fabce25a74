"""Scene-statistic grid construction -- TEST INFRASTRUCTURE ONLY (oracle).

Plain numpy, binary64.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the HIP library never
does, and the two share no code.

It restates Sec. 3.5 (i), Eq. scene-norm and Eq. voxel-size of DivAS (arXiv
2601.04860), with the parameter values of Tab. gs-hyperparams:

  c_scene = coordinate-wise median of the Gaussian centres
  r_fg    = 99th percentile of |mu_i - c_scene|
  b       = ceil(1.05 r_fg)                      (an integer number of scene units)
  h_v     = max(alpha_v * s_med, beta_v * r_fg / g0),  (alpha_v, beta_v, g0) = (3, 1, 256)
  g       = smallest power of two >= 2 b / h_v, capped at g_max
  grid    = the cube of half-extent b around c_scene: origin c_scene - b,
            g voxels of edge 2 b / g per axis

Readings where the paper is silent (each is listed in the design notes):
  - a point takes part iff its three coordinates (and its scale, when scales
    are given) are finite; m counts those points;
  - the median of an even count is the mean of the two middle order
    statistics, (lo + hi) / 2 in binary64;
  - the 99th percentile interpolates linearly between order statistics:
    position q (m - 1), value x_i + (x_{i+1} - x_i) f with i = floor(position)
    and f its fractional part;
  - the distance is sqrt(dx^2 + dy^2 + dz^2) in binary64, summed in that order;
  - r_scene of Eq. voxel-size is r_fg (the only scene radius defined);
  - s_med is the median of one scale per point (the caller's choice, e.g. the
    larger tangent scale of a surfel); without scales the first term is dropped;
  - g is at least 2; the voxel edge is 2 b / g, so the grid covers the cube
    exactly (at the cap the edge exceeds h_v);
  - kept points are those inside the grid by the library's voxel rule
    (floor((mu - origin) / voxel) in [0, g) on every axis).

Parity: the order statistics and the arithmetic above are exact or fixed in
operation order, so the GPU must match every output bit for bit.  Pins:
tests/test_oracle_grid_pins.py (brute-force order statistics, closed-form
scenes, numpy's percentile within rounding, the integer and power-of-two
rules).
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_V, BETA_V, G0, PAD = 3.0, 1.0, 256, 1.05


def order_stat(values, k):
    """The k-th smallest (0-based) of a 1-D float64 array (a library
    partition serves as the selection step)."""
    return float(np.partition(values, k)[k])


def median(values):
    """Median: the middle order statistic, or the mean of the two middle ones."""
    m = len(values)
    if m == 0:
        return math.nan
    if m % 2:
        return order_stat(values, (m - 1) // 2)
    lo = order_stat(values, m // 2 - 1)
    hi = order_stat(values, m // 2)
    return (lo + hi) / 2.0


def percentile_linear(values, q):
    """Percentile q in [0, 1] with linear interpolation between order statistics."""
    m = len(values)
    if m == 0:
        return math.nan
    pos = q * (m - 1)
    i = int(math.floor(pos))
    f = pos - i
    lo = order_stat(values, i)
    if i + 1 >= m:
        return lo
    hi = order_stat(values, i + 1)
    return lo + (hi - lo) * f


def next_pow2_at_least(x, g_max):
    """Smallest power of two g >= x (and >= 2), capped at g_max."""
    g = 2
    while g < x and g < g_max:
        g *= 2
    return min(g, g_max)


def grid_from_points(xyz, scale=None, g_max=512, alpha_v=ALPHA_V, beta_v=BETA_V, g0=G0, pad=PAD):
    """Scene-statistic grid of Eq. scene-norm / Eq. voxel-size.

    xyz: float32 [n, 3] Gaussian centres; scale: float32 [n] or None.
    Returns a dict: center (3 floats), r_fg, b, s_med (nan without scales),
    h_v, dim, origin (3 floats), voxel, m (points taking part), n_kept.
    """
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    use = np.all(np.isfinite(xyz), axis=1)
    if scale is not None:
        scale = np.asarray(scale, dtype=np.float32).reshape(-1)
        use &= np.isfinite(scale)
    p = xyz[use].astype(np.float64)
    m = int(p.shape[0])
    if m == 0:
        raise ValueError("no point with finite coordinates")
    c = [median(p[:, k]) for k in range(3)]
    dx, dy, dz = p[:, 0] - c[0], p[:, 1] - c[1], p[:, 2] - c[2]
    dist = np.sqrt((dx * dx + dy * dy) + dz * dz)
    r_fg = percentile_linear(dist, 0.99)
    b = float(math.ceil(pad * r_fg))
    s_med = median(scale[use].astype(np.float64)) if scale is not None else math.nan
    h_v = beta_v * r_fg / g0
    if scale is not None:
        h_v = max(alpha_v * s_med, h_v)
    if not (b > 0.0) or not (h_v > 0.0):
        raise ValueError("degenerate scene: zero extent")
    dim = next_pow2_at_least(2.0 * b / h_v, g_max)
    origin = [c[k] - b for k in range(3)]
    voxel = 2.0 * b / dim
    # kept: inside the grid by the voxel rule floor((mu - origin) / voxel)
    q = np.floor((xyz.astype(np.float64) - np.asarray(origin)) / voxel)
    kept = np.all((q >= 0) & (q < dim), axis=1)
    return dict(center=c, r_fg=r_fg, b=b, s_med=s_med, h_v=h_v, dim=int(dim), origin=origin, voxel=voxel, m=m,
                n_kept=int(kept.sum()))
