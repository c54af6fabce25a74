"""Needle-floater cull of the voxel-to-surfel mapping -- TEST INFRASTRUCTURE
ONLY (oracle).

Plain numpy, binary64.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the HIP library never
does, and the two share no code.

It restates Pass 2 of the voxel-to-surfel mapping of DivAS (arXiv
2601.04860), Eq. aspect, Eq. needle and Eq. pass-needle:

  a_i   = max(s_i1, s_i2) / (min(s_i1, s_i2) + eps)
  tau_a = 99th percentile of {a_i}
  F2_i  = F1_i and (a_i <= tau_a)

where F1 is the Pass 1 label (the voxel lookup of Eq. pass1).

Readings where the paper is silent (each is listed in the design notes):
  - eps is not given; it is 1e-6, as the fusion's eps;
  - the aspect is evaluated in binary64 from the float32 scales, in the order
    written above;
  - a surfel whose aspect is not finite (a non-finite scale, or a zero
    denominator) stays out of the percentile and is culled;
  - the percentile interpolates linearly between order statistics around
    position 0.99 (m - 1), as in the grid construction.

Parity: bit-exact.  Pins: tests/test_oracle_surfel_pins.py.
"""
from __future__ import annotations

import numpy as np

from .grid_stats import percentile_linear

EPS = 1e-6


def aspect(scales, eps=EPS):
    """Eq. aspect per surfel; NaN where it is not finite."""
    s = np.asarray(scales, dtype=np.float32).reshape(-1, 2).astype(np.float64)
    hi = np.maximum(s[:, 0], s[:, 1])
    lo = np.minimum(s[:, 0], s[:, 1])
    with np.errstate(divide="ignore", invalid="ignore"):
        a = hi / (lo + eps)
    ok = np.all(np.isfinite(s), axis=1) & np.isfinite(a)
    return np.where(ok, a, np.nan)


def needle_threshold(scales, q=0.99, eps=EPS):
    """Eq. needle: tau_a over the surfels with an aspect."""
    a = aspect(scales, eps)
    a = a[np.isfinite(a)]
    if a.size == 0:
        raise ValueError("no surfel has finite scales")
    return percentile_linear(a, q)


def needle_cull(labels, scales, eps=EPS):
    """Eq. pass-needle.  Returns (F2 uint8 labels, tau_a, number of surfels
    with a > tau_a or no aspect)."""
    labels = np.asarray(labels, dtype=np.uint8).reshape(-1)
    a = aspect(scales, eps)
    tau = needle_threshold(scales, eps=eps)
    keep = np.isfinite(a) & (a <= tau)
    out = (labels & keep.astype(np.uint8)).astype(np.uint8)
    return out, tau, int((~keep).sum())
