"""The allocation-free needle cull (divas_needle_cull_noalloc) through the C
ABI against the allocating entry point divas_needle_cull on the same inputs:
threshold, culled count and labels bit-exact, on two calls in a row (the
second smaller, so whatever the first left in the fixed scratch must not
leak into it), plus the oracle on the smaller one and the size limit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2601_04860_amd as dv  # noqa: E402
from oracle import surfel_map as S  # noqa: E402
from tests import _helpers as H  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scales(n, seed):
    """Two log-normal tangent scales per surfel, 1% stretched into needles."""
    rng = np.random.default_rng(seed)
    s = np.exp(0.5 * rng.standard_normal((n, 2))) * 0.01
    k = rng.random(n) < 0.01
    s[k, 0] *= np.exp(rng.random(k.sum()) * 8)
    return s.astype(np.float32)


def _both(ctx, n, seed, oracle_check):
    _say(f"[case] needle noalloc n={n} seed={seed}")
    rng = np.random.default_rng(seed)
    lab = (rng.random(n) < 0.6).astype(np.uint8)
    sc = _scales(n, seed)
    if n > 1000:
        sc[::997, 0] = np.nan                  # a few surfels without an aspect
    scd = H.to_dev(sc)
    lab_a = H.to_dev(lab)
    lab_b = H.to_dev(lab)
    tau_a, cut_a = dv.needle_cull(ctx, scd, lab_a)
    tau_b, cut_b = dv.needle_cull_noalloc(ctx, scd, lab_b)
    assert tau_b == tau_a and cut_b == cut_a, ((tau_b, cut_b), (tau_a, cut_a))
    got = lab_b.cpu().numpy()
    assert np.array_equal(got, lab_a.cpu().numpy())
    if oracle_check:
        ref, tau_ref, cut_ref = S.needle_cull(lab, sc)
        assert tau_b == tau_ref and cut_b == cut_ref
        assert np.array_equal(got, ref)
    _say(f"[ok] needle noalloc n={n}: tau={tau_b:.6g} culled={cut_b}")


def test_noalloc_needle_cull_equals_the_allocating_call():
    ctx = dv.Context(0)
    # the largest input first, then a smaller one on the same fixed scratch
    _both(ctx, dv.NOALLOC_MAX_SURFELS, 41, oracle_check=False)
    _both(ctx, 123_457, 42, oracle_check=True)
    _both(ctx, 1, 43, oracle_check=True)


def test_noalloc_needle_cull_rejects_more_than_its_maximum():
    ctx = dv.Context(0)
    n = dv.NOALLOC_MAX_SURFELS + 1
    _say(f"[case] needle noalloc over the maximum: n={n}")
    lab = H.to_dev(np.ones(n, np.uint8))
    with pytest.raises(dv.DivasError) as ei:
        dv.needle_cull_noalloc(ctx, H.to_dev(np.ones((n, 2), np.float32)), lab)
    assert ei.value.status == dv.ERR_CAPACITY
    with pytest.raises(dv.DivasError):
        dv.needle_cull_noalloc(ctx, H.to_dev(np.ones((4, 2), np.float32)), H.to_dev(np.ones(4, np.uint8)), eps=-1.0)
    assert bool(lab.cpu().numpy().all())
    _say("[ok] needle noalloc over the maximum rejected")
