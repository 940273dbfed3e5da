"""Point selection before registration (Sec. IV, considerations for performance:
FAST corners, no non-maximum suppression, threshold chosen automatically so
that a few thousand pixels with depth are kept) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library never does.

Plain numpy, written from the definitions:
  * FAST segment test (Rosten and Drummond, 2006): pixel p with intensity I_p
    is a corner at threshold t if some arc of at least 9 contiguous pixels of
    the 16-pixel circle of radius 3 around p is all brighter than I_p + t or
    all darker than I_p - t.  Pixels closer than 3 to the border are never
    tested.
  * Score of p: the largest integer t at which p is a corner (-1 if none).
    An arc A is all brighter at t iff min_A I > I_p + t, i.e. for every
    t <= min_A I - I_p - 1, and all darker iff t <= I_p - max_A I - 1, so the
    score is the maximum of those bounds over the 16 arcs of 9.
  * Threshold: the count of corners with valid depth is non-increasing in t;
    the threshold is the smallest t whose count does not exceed the cap, so
    the selection is as large as the cap allows.
  * Selected pixels in raster order, back-projected through the pinhole
    model: z = depth, x = (u - cx) z / fx, y = (v - cy) z / fy (FP64, then
    rounded to FP32); their feature rows are copied unchanged.
"""
from __future__ import annotations

import numpy as np

# Bresenham circle of radius 3, as (du, dv) offsets, in circular order
CIRCLE = ((0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
          (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3))
ARC = 9


def fast_scores(gray):
    """Per-pixel score (int32, H x W): the largest threshold at which the
    pixel passes the 9-of-16 segment test, -1 if it passes at no threshold
    or lies within 3 pixels of the border."""
    g = np.asarray(gray).astype(np.int32)
    H, W = g.shape
    s = np.full((H, W), -1, np.int32)
    if H < 7 or W < 7:
        return s
    c = g[3:H - 3, 3:W - 3]
    ring = np.stack([g[3 + dv:H - 3 + dv, 3 + du:W - 3 + du] for du, dv in CIRCLE])
    best = np.full(c.shape, -1, np.int32)
    for k in range(16):
        arc = ring[[(k + j) % 16 for j in range(ARC)]]
        bright = arc.min(axis=0) - c - 1
        dark = c - arc.max(axis=0) - 1
        best = np.maximum(best, np.maximum(bright, dark))
    s[3:H - 3, 3:W - 3] = best
    return s


def valid_depth(depth, camera):
    d = np.asarray(depth, np.float32)
    with np.errstate(invalid="ignore"):
        return np.isfinite(d) & (d >= np.float32(camera["depth_min"])) & (d <= np.float32(camera["depth_max"]))


def select_threshold(score, valid, max_points):
    """(t, count): the smallest t in [0, 255] with #{valid, score >= t} <=
    max_points (t = 255 keeps nothing, as scores are at most 254)."""
    for t in range(256):
        n = int(np.count_nonzero(valid & (score >= t)))
        if n <= max_points:
            return t, n
    raise AssertionError("unreachable: no score reaches 255")


def select_points(gray, depth, feat, camera, max_points):
    """Returns (xyz float32 n x 3, feat float32 n x D, threshold, pixel indices
    in raster order, scores)."""
    score = fast_scores(gray)
    valid = valid_depth(depth, camera)
    t, n = select_threshold(score, valid, max_points)
    H, W = score.shape
    idx = np.flatnonzero((valid & (score >= t)).ravel())
    assert idx.size == n
    u = (idx % W).astype(np.float64)
    v = (idx // W).astype(np.float64)
    z = np.asarray(depth, np.float32).ravel()[idx].astype(np.float64)
    x = ((u - camera["cx"]) * z) / camera["fx"]
    y = ((v - camera["cy"]) * z) / camera["fy"]
    xyz = np.stack([x, y, z], axis=1).astype(np.float32)
    D = 0 if feat is None else feat.shape[-1]
    f = np.zeros((n, 0), np.float32) if D == 0 else np.asarray(feat, np.float32).reshape(H * W, D)[idx]
    return xyz, f, t, idx, score
