"""Pins of the point-selection oracle (FAST segment test with an automatic
threshold, Sec. IV's performance considerations) against what the definition
fixes: a literal run-length segment test on small images, hand-built circle
patterns, the monotone count behind the threshold, and the pinhole
back-projection."""
import numpy as np
import pytest

import oracle
from oracle.select import CIRCLE


def _segment_test(g, v, u, t):
    """Literal FAST test: label the 16 circle pixels brighter (> I_p + t),
    darker (< I_p - t) or similar, and look for a circular run of >= 9 equal
    non-similar labels."""
    p = int(g[v, u])
    lab = []
    for du, dv in CIRCLE:
        q = int(g[v + dv, u + du])
        lab.append(1 if q > p + t else (-1 if q < p - t else 0))
    for want in (1, -1):
        run = 0
        for k in range(32):  # twice around the circle for wrapped runs
            run = run + 1 if lab[k % 16] == want else 0
            if run >= 9:
                return True
    return False


@pytest.mark.parametrize("seed", range(4))
def test_score_equals_literal_segment_test(seed):
    """score(p) >= t exactly when the literal segment test passes at t, for
    every interior pixel and every t in 0..255, on images with few grey levels
    (long equal-label runs, exact ties at the threshold)."""
    rng = np.random.default_rng(seed)
    g = rng.choice(np.array([0, 40, 41, 90, 160, 200, 255], np.uint8), size=(12, 13))
    g[4:8, 4:9] = 160  # a flat patch with corners
    s = oracle.fast_scores(g)
    H, W = g.shape
    for v in range(H):
        for u in range(W):
            if v < 3 or u < 3 or v >= H - 3 or u >= W - 3:
                assert s[v, u] == -1
                continue
            passes = [_segment_test(g, v, u, t) for t in range(256)]
            # the literal test is monotone in t, and the score is where it stops
            assert all(not b or a for a, b in zip(passes, passes[1:]))
            assert s[v, u] == (max(t for t in range(256) if passes[t]) if passes[0] else -1)


def _ring_image(centre, ring_values):
    g = np.full((7, 7), centre, np.uint8)
    for (du, dv), q in zip(CIRCLE, ring_values):
        g[3 + dv, 3 + du] = q
    return g


def test_hand_built_circle_patterns():
    # uniform: never a corner
    assert (oracle.fast_scores(np.full((9, 9), 77, np.uint8)) == -1).all()
    # dark centre under a uniform bright ring: every arc is brighter by 200
    assert oracle.fast_scores(_ring_image(0, [200] * 16))[3, 3] == 199
    # 9 contiguous pixels brighter by 50 (wrapping past the start), 7 equal
    ring = [150] * 16
    for k in range(12, 21):
        ring[k % 16] = 200
    assert oracle.fast_scores(_ring_image(150, ring))[3, 3] == 49
    # only 8 brighter: no arc of 9 at any threshold
    ring[20 % 16] = 150
    assert oracle.fast_scores(_ring_image(150, ring))[3, 3] == -1
    # 9 darker by 30 except one pixel only 10 darker: the weakest pixel bounds the arc
    ring = [100] * 16
    for k in range(9):
        ring[k] = 70
    ring[4] = 90
    assert oracle.fast_scores(_ring_image(100, ring))[3, 3] == 9
    # too small to hold an interior pixel
    assert (oracle.fast_scores(np.zeros((6, 40), np.uint8)) == -1).all()


def test_threshold_is_smallest_under_the_cap():
    rng = np.random.default_rng(7)
    g = rng.integers(0, 256, size=(40, 50)).astype(np.uint8)
    depth = rng.uniform(0.5, 6.0, size=g.shape).astype(np.float32)
    depth[rng.random(g.shape) < 0.2] = 0.0
    cam = dict(fx=50.0, fy=55.0, cx=24.5, cy=19.5, depth_min=1.0, depth_max=5.0)
    s = oracle.fast_scores(g)
    valid = oracle.valid_depth(depth, cam)
    counts = [int(np.count_nonzero(valid & (s >= t))) for t in range(256)]
    assert all(a >= b for a, b in zip(counts, counts[1:])) and counts[255] == 0
    for cap in (0, 1, 10, 100, counts[0], counts[0] + 5):
        t, n = oracle.select_threshold(s, valid, cap)
        assert n == counts[t] <= cap
        assert t == 0 or counts[t - 1] > cap


def test_back_projection_closed_form():
    rng = np.random.default_rng(3)
    H, W = 30, 40
    g = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    depth = rng.uniform(2.0, 3.0, size=(H, W)).astype(np.float32)
    feat = rng.random((H, W, 4)).astype(np.float32)
    cam = dict(fx=30.0, fy=32.0, cx=20.0, cy=15.0, depth_min=0.1, depth_max=10.0)
    xyz, f, t, idx, s = oracle.select_points(g, depth, feat, cam, 10 ** 6)
    assert t == 0 and np.array_equal(idx, np.flatnonzero((s >= 0).ravel()))
    u, v = idx % W, idx // W
    # reprojection through the pinhole recovers the pixel; depth is z
    np.testing.assert_allclose(cam["fx"] * xyz[:, 0] / xyz[:, 2] + cam["cx"], u, atol=1e-4)
    np.testing.assert_allclose(cam["fy"] * xyz[:, 1] / xyz[:, 2] + cam["cy"], v, atol=1e-4)
    np.testing.assert_array_equal(xyz[:, 2], depth.ravel()[idx])
    np.testing.assert_array_equal(f, feat.reshape(H * W, 4)[idx])
    on_axis = (u == 20) & (v == 15)
    assert (xyz[on_axis, :2] == 0).all()
