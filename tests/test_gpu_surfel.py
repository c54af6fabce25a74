"""GPU parity of the needle-floater cull (Pass 2 of the voxel-to-surfel
mapping; Eq. aspect, Eq. needle, Eq. pass-needle) through the C ABI against
the oracle: threshold, culled count and labels bit-exact."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2601_04860_amd as dv  # noqa: E402
import scenes  # noqa: E402
from oracle import surfel_map as S  # noqa: E402
from tests import _helpers as H  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dv.Context(0)


def _scales(n, seed, needles=0.01):
    """Two log-normal tangent scales per surfel, a fraction stretched into needles."""
    rng = np.random.default_rng(seed)
    s = np.exp(0.5 * rng.standard_normal((n, 2))) * 0.01
    k = rng.random(n) < needles
    s[k, 0] *= np.exp(rng.random(k.sum()) * 8)
    return s.astype(np.float32)


def _check(ctx, name, labels, scales):
    _say(f"[case] needle {name}: n={len(labels)}")
    ref, tau_ref, cut_ref = S.needle_cull(labels, scales)
    lab = H.to_dev(labels.astype(np.uint8))
    tau, cut = dv.needle_cull(ctx, H.to_dev(scales), lab)
    assert tau == tau_ref, (tau, tau_ref)
    assert cut == cut_ref, (cut, cut_ref)
    assert np.array_equal(lab.cpu().numpy(), ref)
    _say(f"[ok] needle {name}: tau={tau:.6g} culled={cut}")


def test_needle_cull_after_pass1_labels(ctx):
    """c1 end to end: fusion, Pass 1 labels of the points, then Pass 2."""
    s = scenes.config_scene("c1")
    lp = H.lib_params(s.voxel)
    _, sess = H.make_session(s, lp, ctx=ctx)
    sess.fuse_views(H.upload_views(s.views))
    pts = np.asarray(s.points, np.float32)
    lab = sess.label_points(H.to_dev(pts)).cpu().numpy()
    assert lab.any()
    _check(ctx, "c1 pass 1 + 2", lab, _scales(len(pts), 3))
    sess.close()


def test_needle_cull_sizes_and_special_values(ctx):
    rng = np.random.default_rng(17)
    for n in (1, 2, 100, 4097, 3_000_000):
        lab = (rng.random(n) < 0.6).astype(np.uint8)
        _check(ctx, f"n={n}", lab, _scales(n, n))
    sc = _scales(5000, 5)
    sc[::37, 0] = np.nan
    sc[5::41, 1] = np.inf
    sc[9::53] = 0.0                       # aspect 0 / eps = 0
    sc[11::59, 1] = -sc[11::59, 1]        # negative scales still give a finite aspect
    _check(ctx, "special", np.ones(5000, np.uint8), sc)
    # equal aspects everywhere: nothing is above the threshold
    _check(ctx, "flat", np.ones(999, np.uint8), np.ones((999, 2), np.float32))


def test_needle_cull_rejects_bad_inputs(ctx):
    lab = H.to_dev(np.ones(4, np.uint8))
    with pytest.raises(dv.DivasError):
        dv.needle_cull(ctx, H.to_dev(np.full((4, 2), np.nan, np.float32)), lab)
    with pytest.raises(dv.DivasError):
        dv.needle_cull(ctx, H.to_dev(np.ones((4, 2), np.float32)), lab, eps=-1.0)
    assert np.all(lab.cpu().numpy() == 1)
