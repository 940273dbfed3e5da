"""Seeded synthetic point-cloud pairs shaped like the paper's workloads.

The paper evaluates on KITTI stereo odometry and TUM RGB-D (Sec. V); neither
dataset, nor the depth and semantic networks it uses, is available, so these
generators stand in for them with the same shapes: a pinhole camera grid,
depth ranges, depth noise growing with depth squared, colour-like and
class-probability features, and a known relative motion between the two
frames.  This module holds input generation only -- no part of the
registration arithmetic -- and is shared by the tests, the benchmark and the
oracle inputs.  Rotations come from ``scipy.spatial.transform``.

Conventions: camera frame x right, y down, z forward.  ``T_gt`` (4x4, float64)
maps coordinates of the second cloud Z into the frame of the first cloud X,
so the registration maximiser is T ~= T_gt.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation


def se_block(dim, ell, sigma=1.0):
    """Squared-exponential feature block (eq. (5))."""
    return {"kind": "se", "dim": int(dim), "ell": float(ell), "sigma": float(sigma)}


def lin_block(dim):
    """Linear (inner-product) feature block (eq. (4), (6))."""
    return {"kind": "lin", "dim": int(dim), "ell": 1.0, "sigma": 1.0}


@dataclass
class Pair:
    name: str
    x: np.ndarray          # N x 3 float32
    u: np.ndarray          # N x D float32
    z: np.ndarray          # M x 3 float32
    v: np.ndarray          # M x D float32
    spec: list
    T_gt: np.ndarray       # 4 x 4 float64
    ell: float             # lengthscale for single evaluations
    align: dict = field(default_factory=dict)
    T_eval: np.ndarray = None  # pose for single evaluations (defaults to identity)

    @property
    def D(self):
        return int(sum(b["dim"] for b in self.spec))


def _rigid(R, t):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def _unit(rng):
    a = rng.normal(size=3)
    return a / np.linalg.norm(a)


def _apply(T, p):
    return p @ T[:3, :3].T + T[:3, 3]


def _inv(T):
    R = T[:3, :3]
    return _rigid(R.T, -R.T @ T[:3, 3])


def random_motion(rng, angle_deg, trans_m):
    R = Rotation.from_rotvec(np.deg2rad(angle_deg) * _unit(rng)).as_matrix()
    return _rigid(R, trans_m * _unit(rng))


# ---------------------------------------------------------------- textures
def _texture(pw, freq, phase):
    """Three colour-like channels in [0,1], functions of world position."""
    arg = pw @ freq.T + phase                         # n x 6
    c = 0.5 + 0.25 * (np.sin(arg[:, 0:3]) + np.sin(arg[:, 3:6]))
    return np.clip(c, 0.0, 1.0)


def _texture_grad(pw, normal, freq, phase):
    """Two tangent-plane derivatives of the mean channel, mapped to [0,1]."""
    arg = pw @ freq.T + phase
    # d/dp of mean_k 0.25 (sin(a_k.p) + sin(b_k.p))
    g = 0.25 / 3.0 * (np.cos(arg[:, 0:3]) @ freq[0:3] + np.cos(arg[:, 3:6]) @ freq[3:6])
    ref = np.where(np.abs(normal[:, 1:2]) > 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(normal, ref)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(normal, t1)
    scale = 1.0 / (np.abs(freq).sum() / 6.0 + 1e-9)
    g1 = 0.5 + 0.5 * np.tanh(scale * np.sum(g * t1, axis=1))
    g2 = 0.5 + 0.5 * np.tanh(scale * np.sum(g * t2, axis=1))
    return np.stack([g1, g2], axis=1)


def _colour_features(rng, pw, normal, freq, phase):
    f = np.concatenate([_texture(pw, freq, phase), _texture_grad(pw, normal, freq, phase)], axis=1)
    return np.clip(f + rng.normal(0.0, 0.01, f.shape), 0.0, 1.0)


# ---------------------------------------------------------------- ray casting
class _Scene:
    """Planes (point on plane, normal) and axis-aligned boxes (lo, hi)."""

    def __init__(self):
        self.planes = []
        self.boxes = []

    def cast(self, o, d, with_id=False):
        """Nearest hit along rays o + t d (t > 0). Returns t, normal (inf where
        none) and, if asked, the index of the surface hit (planes first, then
        boxes; -1 where none)."""
        n = d.shape[0]
        best = np.full(n, np.inf)
        nrm = np.zeros((n, 3))
        oid = np.full(n, -1)
        for k, (p0, nv) in enumerate(self.planes):
            den = d @ nv
            with np.errstate(divide="ignore", invalid="ignore"):
                t = ((p0 - o) @ nv) / den
            ok = (np.abs(den) > 1e-12) & (t > 1e-6) & (t < best)
            best[ok] = t[ok]
            nrm[ok] = nv
            oid[ok] = k
        for k, (lo, hi) in enumerate(self.boxes):
            with np.errstate(divide="ignore", invalid="ignore"):
                inv = 1.0 / d
                t0 = (lo - o) * inv
                t1 = (hi - o) * inv
            tmin = np.minimum(t0, t1)
            tmax = np.maximum(t0, t1)
            tin = np.nanmax(tmin, axis=1)
            tout = np.nanmin(tmax, axis=1)
            ok = (tin <= tout) & (tin > 1e-6) & (tin < best)
            if np.any(ok):
                best[ok] = tin[ok]
                ax = np.argmax(tmin[ok], axis=1)
                nn = np.zeros((ok.sum(), 3))
                nn[np.arange(ok.sum()), ax] = 1.0
                nrm[ok] = nn
                oid[ok] = len(self.planes) + k
        return (best, nrm, oid) if with_id else (best, nrm)


def _render(rng, scene, cam, width, height, f, cx, cy, npts, dmin, dmax, noise_k,
            freq, phase, semantic_dim=0, stride=1, lazy=False):
    """Sample npts pixels with valid depth; return camera-frame points and features.
    lazy: cast rays only through a random subset of pixels, drawn in batches
    until npts of them have valid depth (the same distribution -- a uniform
    sample of the valid pixels -- at a fraction of the cost; another random
    stream than the full cast)."""
    us, vs = np.meshgrid(np.arange(0, width, stride), np.arange(0, height, stride))
    us = us.reshape(-1).astype(np.float64)
    vs = vs.reshape(-1).astype(np.float64)
    dc = np.stack([(us - cx) / f, (vs - cy) / f, np.ones_like(us)], axis=1)
    R, t = cam[:3, :3], cam[:3, 3]
    if lazy:
        order = rng.permutation(us.size)
        got, start, step = [], 0, max(1024, int(1.25 * npts))
        depth = np.full(us.size, np.inf)
        nrm = np.zeros((us.size, 3))
        dw = np.zeros_like(dc)
        while sum(g.size for g in got) < npts and start < us.size:
            idx = order[start:start + step]
            start += idx.size
            dw[idx] = dc[idx] @ R.T
            depth[idx], nrm[idx] = scene.cast(np.broadcast_to(t, (idx.size, 3)), dw[idx])
            d_i = depth[idx]
            got.append(idx[np.isfinite(d_i) & (d_i >= dmin) & (d_i <= dmax)])
            step = max(1024, int(1.25 * (npts - sum(g.size for g in got))))
        valid = np.concatenate(got) if got else np.zeros(0, np.int64)
        if valid.size < npts:
            raise ValueError(f"only {valid.size} valid pixels for {npts} requested")
        pick = np.sort(valid[:npts])
        o = np.broadcast_to(t, dw.shape)
    else:
        dw = dc @ R.T
        o = np.broadcast_to(t, dw.shape)
        depth, nrm = scene.cast(o, dw)
        valid = np.flatnonzero(np.isfinite(depth) & (depth >= dmin) & (depth <= dmax))
        if valid.size < npts:
            raise ValueError(f"only {valid.size} valid pixels for {npts} requested")
        pick = np.sort(rng.choice(valid, size=npts, replace=False))
    dep = depth[pick]
    pw = o[pick] + dep[:, None] * dw[pick]
    noisy = dep + rng.normal(0.0, 1.0, npts) * noise_k * dep * dep
    pc = noisy[:, None] * dc[pick]
    feats = [_colour_features(rng, pw, nrm[pick], freq, phase)]
    if semantic_dim:
        feats.append(rng.dirichlet(np.full(semantic_dim, 0.3), size=npts))
    return pc, np.concatenate(feats, axis=1)


def _stereo_scene(rng):
    s = _Scene()
    s.planes.append((np.array([0.0, 1.65, 0.0]), np.array([0.0, 1.0, 0.0])))   # ground
    s.planes.append((np.array([-7.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0])))   # left facade
    s.planes.append((np.array([9.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0])))    # right facade
    for _ in range(30):
        size = rng.uniform(0.5, 4.0, 3)
        c = np.array([rng.uniform(-6.0, 8.0), 1.65 - size[1] / 2.0, rng.uniform(5.0, 40.0)])
        s.boxes.append((c - size / 2.0, c + size / 2.0))
    return s


def _room_scene(rng):
    s = _Scene()
    lo = np.array([-3.0, -1.8, -0.5])
    hi = np.array([3.0, 1.2, 3.5])
    for ax in range(3):
        nv = np.zeros(3); nv[ax] = 1.0
        s.planes.append((lo.copy(), nv))
        s.planes.append((hi.copy(), nv))
    for _ in range(8):
        size = rng.uniform(0.2, 1.2, 3)
        c = np.array([rng.uniform(-2.4, 2.4), 1.2 - size[1] / 2.0, rng.uniform(0.8, 3.0)])
        s.boxes.append((c - size / 2.0, c + size / 2.0))
    return s


def _tex_params(rng, wavelength):
    freq = rng.normal(size=(6, 3))
    freq *= (2.0 * np.pi / wavelength) / np.linalg.norm(freq, axis=1, keepdims=True)
    return freq, rng.uniform(0, 2 * np.pi, 6)


def _shuffle(rng, p, f):
    perm = rng.permutation(p.shape[0])
    return p[perm], f[perm]


# ---------------------------------------------------------------- workloads
def tiny_cube(seed=1000, n=2000):
    """2,000 points uniform in a 4 m cube, 5 colour features U[0,1];
    Z = T_gt^-1 X + N(0, 0.01 m), T_gt = 5 deg about a random axis, 0.1 m."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-2.0, 2.0, (n, 3))
    u = rng.uniform(0.0, 1.0, (n, 5))
    T_gt = random_motion(rng, 5.0, 0.1)
    z = _apply(_inv(T_gt), x) + rng.normal(0.0, 0.01, x.shape)
    z, v = _shuffle(rng, z, u)
    return Pair("tiny_cube", x.astype(np.float32), u.astype(np.float32), z.astype(np.float32),
                v.astype(np.float32), [se_block(5, 0.2)], T_gt, 0.1,
                align=dict(ell_init=0.1, ell_min=0.1, max_iter=50, fixed_iters=True))


def stereo_pair(seed=1001, n=30000, m=None, motion=None, semantic=True, ell_init=0.95,
                ell_min=0.1, lazy=False):
    """KITTI-stereo-shaped pair: 1241x376 grid, f=700, depth 2-40 m, ground,
    facades and 30 boxes, depth noise 5e-4 d^2, 5 colour+gradient features and
    (optionally) a 19-class Dirichlet(0.3) probability vector."""
    rng = np.random.default_rng(seed)
    m = n if m is None else m
    scene = _stereo_scene(rng)
    freq, phase = _tex_params(rng, 3.0)
    if motion is None:
        R = Rotation.from_rotvec(np.deg2rad(2.0) * np.array([0.0, 1.0, 0.0])).as_matrix()
        C2 = _rigid(R, np.array([0.0, 0.0, 1.0]))
    else:
        C2 = motion
    sem = 19 if semantic else 0
    x, u = _render(rng, scene, np.eye(4), 1241, 376, 700.0, 620.0, 188.0, n, 2.0, 40.0, 5e-4,
                   freq, phase, sem, lazy=lazy)
    z, v = _render(rng, scene, C2, 1241, 376, 700.0, 620.0, 188.0, m, 2.0, 40.0, 5e-4,
                   freq, phase, sem, lazy=lazy)
    spec = [se_block(5, 0.2)] + ([lin_block(19)] if semantic else [])
    return Pair("stereo", x.astype(np.float32), u.astype(np.float32), z.astype(np.float32),
                v.astype(np.float32), spec, C2, ell_init,
                align=dict(ell_init=ell_init, ell_min=ell_min, max_iter=4000))


@dataclass
class Sequence:
    """Frames of one camera moving through a scene: frame k is (xyz, features)
    in camera k's frame; poses[k] maps camera k into the world (frame 0 = I)."""
    name: str
    frames: list
    spec: list
    poses: list
    first: dict            # ascent parameters of the first pair (from identity)
    rest: dict             # ascent parameters of later pairs (warm-started)

    def relative(self, k):
        """Ground-truth pose of frame k + 1 in frame k's coordinates."""
        return _inv(self.poses[k]) @ self.poses[k + 1]

    def drift(self, rel):
        """End-point drift of estimated relative poses (see trajectory_drift)."""
        return trajectory_drift(self.poses, rel)


def trajectory_drift(poses, rel):
    """End-point drift of estimated relative poses rel[k] (frame k + 1 in
    frame k) chained from frame 0, against the true poses: translation error
    in % of the path length and rotation error in deg per m."""
    T = np.eye(4)
    for R in rel:
        T = T @ R
    E = _inv(poses[len(rel)]) @ T
    path = sum(np.linalg.norm((_inv(poses[k]) @ poses[k + 1])[:3, 3]) for k in range(len(rel)))
    ang = np.degrees(np.arccos(np.clip((np.trace(E[:3, :3]) - 1.0) / 2.0, -1.0, 1.0)))
    return 100.0 * np.linalg.norm(E[:3, 3]) / path, ang / path


def stereo_sequence(seed=1005, frames=8, n=30000, step=1.0, yaw_deg=2.0, semantic=True):
    """Frame-to-frame sequence in the stereo-outdoor scene: the camera moves
    `step` m (+-20%) along its optical axis per frame and turns `yaw_deg`
    (+-30%) about its vertical axis; every frame samples its own pixels among
    the hits of every second pixel row and column (depth noise 5e-4 d^2).  The
    first pair starts at the identity with
    ell 0.95 -> 0.1, later pairs at the previous estimate with ell 0.1."""
    rng = np.random.default_rng(seed)
    scene = _stereo_scene(rng)
    freq, phase = _tex_params(rng, 3.0)
    poses = [np.eye(4)]
    for _ in range(frames - 1):
        yaw = np.deg2rad(yaw_deg) * (1.0 + 0.3 * rng.uniform(-1.0, 1.0))
        fwd = step * (1.0 + 0.2 * rng.uniform(-1.0, 1.0))
        R = Rotation.from_rotvec(yaw * np.array([0.0, 1.0, 0.0])).as_matrix()
        poses.append(poses[-1] @ _rigid(R, np.array([0.0, 0.0, fwd])))
    sem = 19 if semantic else 0
    out = []
    for P in poses:
        x, u = _render(rng, scene, P, 1241, 376, 700.0, 620.0, 188.0, n, 2.0, 40.0, 5e-4, freq, phase, sem,
                       stride=2)
        out.append((x.astype(np.float32), u.astype(np.float32)))
    spec = [se_block(5, 0.2)] + ([lin_block(19)] if semantic else [])
    return Sequence("stereo_sequence", out, spec, poses,
                    first=dict(ell_init=0.95, ell_min=0.1, max_iter=4000),
                    rest=dict(ell_init=0.1, ell_min=0.1, max_iter=4000))


@dataclass
class ImageFrame:
    gray: np.ndarray    # H x W uint8 intensity
    depth: np.ndarray   # H x W float32 (m); 0 where the pixel has no depth
    feat: np.ndarray    # H x W x D float32 per-pixel features


@dataclass
class ImageSequence:
    name: str
    frames: list        # [ImageFrame]
    camera: dict        # fx, fy, cx, cy, depth_min, depth_max
    spec: list
    poses: list         # camera k -> world, 4 x 4

    def relative(self, k):
        """True pose of frame k + 1 in frame k (maps Z coordinates into X's frame)."""
        return _inv(self.poses[k]) @ self.poses[k + 1]


def stereo_images(seed=1006, frames=2, step=1.0, yaw_deg=2.0, semantic=True, width=1241, height=376):
    """Full-resolution frames of the stereo-outdoor scene for point selection.
    Camera as in stereo_pair (f = 700, c = (620, 188)); the camera moves `step`
    m (+-20%) forward and turns `yaw_deg` (+-30%) per frame along a road kept
    free of boxes (|x| < 3 m).  Grey level =
    255 x surface albedo (U[0.25, 0.9] per plane or box) x (0.55 or 1.0 on a
    0.7 m-wavelength checker pattern of two plane waves in world coordinates)
    + N(0, 1.5), sky 235 + N(0, 1.5), rounded and
    clipped to uint8.  Depth: ray length along z with noise 5e-4 d^2, 0 where
    there is no hit.  Features: 5 colour/gradient channels (3 m texture, as in
    stereo_pair) + 19 Dirichlet(0.3) class probabilities, zero without a hit."""
    rng = np.random.default_rng(seed)
    scene = _stereo_scene(rng)
    # a clear road: boxes reaching into |x| < 3 m would stand in the camera's path
    scene.boxes = [b for b in scene.boxes if b[1][0] <= -3.0 or b[0][0] >= 3.0]
    freq, phase = _tex_params(rng, 3.0)
    gfreq, gphase = _tex_params(rng, 0.7)
    albedo = rng.uniform(0.25, 0.9, len(scene.planes) + len(scene.boxes))
    f, cx, cy = 700.0, 620.0, 188.0
    poses = [np.eye(4)]
    for _ in range(frames - 1):
        yaw = np.deg2rad(yaw_deg) * (1.0 + 0.3 * rng.uniform(-1.0, 1.0))
        fwd = step * (1.0 + 0.2 * rng.uniform(-1.0, 1.0))
        R = Rotation.from_rotvec(yaw * np.array([0.0, 1.0, 0.0])).as_matrix()
        poses.append(poses[-1] @ _rigid(R, np.array([0.0, 0.0, fwd])))
    us, vs = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    dc = np.stack([(us.ravel() - cx) / f, (vs.ravel() - cy) / f, np.ones(us.size)], axis=1)
    sem = 19 if semantic else 0
    out = []
    for P in poses:
        dw = dc @ P[:3, :3].T
        o = np.broadcast_to(P[:3, 3], dw.shape)
        dep, nrm, oid = scene.cast(o, dw, with_id=True)
        hit = np.isfinite(dep)
        pw = o[hit] + dep[hit, None] * dw[hit]
        arg = pw @ gfreq[:2].T + gphase[:2]
        shade = 0.55 + 0.45 * ((np.sin(arg[:, 0]) > 0) ^ (np.sin(arg[:, 1]) > 0))
        g = np.full(us.size, 235.0)
        g[hit] = 255.0 * albedo[oid[hit]] * shade
        g += rng.normal(0.0, 1.5, us.size)
        gray = np.clip(np.rint(g), 0, 255).astype(np.uint8).reshape(height, width)
        d = np.zeros(us.size)
        d[hit] = dep[hit] + rng.normal(0.0, 1.0, hit.sum()) * 5e-4 * dep[hit] ** 2
        feat = np.zeros((us.size, 5 + sem), np.float32)
        feat[hit, :5] = _colour_features(rng, pw, nrm[hit], freq, phase)
        if sem:
            feat[hit, 5:] = rng.dirichlet(np.full(sem, 0.3), size=int(hit.sum()))
        out.append(ImageFrame(gray, d.astype(np.float32).reshape(height, width),
                              feat.reshape(height, width, 5 + sem)))
    spec = [se_block(5, 0.2)] + ([lin_block(19)] if semantic else [])
    cam = dict(fx=f, fy=f, cx=cx, cy=cy, depth_min=2.0, depth_max=40.0)
    return ImageSequence("stereo_images", out, cam, spec, poses)


def rgbd_pair(seed=1002, n=40000, m=None, motion=None, ell_init=0.1, ell_min=0.05, lazy=False):
    """TUM-RGB-D-shaped pair: 640x480 grid, f=525, box room 6x4x3 m with 8
    cuboids, depth 0.5-5 m, noise 0.005 d^2, 5 colour+gradient features;
    motion 3 deg about a random axis and 0.05 m."""
    rng = np.random.default_rng(seed)
    m = n if m is None else m
    scene = _room_scene(rng)
    freq, phase = _tex_params(rng, 0.8)
    C2 = random_motion(rng, 3.0, 0.05) if motion is None else motion
    x, u = _render(rng, scene, np.eye(4), 640, 480, 525.0, 319.5, 239.5, n, 0.5, 5.0, 0.005,
                   freq, phase, lazy=lazy)
    z, v = _render(rng, scene, C2, 640, 480, 525.0, 319.5, 239.5, m, 0.5, 5.0, 0.005,
                   freq, phase, lazy=lazy)
    return Pair("rgbd", x.astype(np.float32), u.astype(np.float32), z.astype(np.float32),
                v.astype(np.float32), [se_block(5, 0.2)], C2, ell_init,
                align=dict(ell_init=ell_init, ell_min=ell_min, max_iter=4000))


def learned_batch(seed=1003, batch=8, n=10000):
    """Stereo-shaped pairs with 32-dim L2-normalised N(0,1) features (LIN kernel),
    evaluated at T = T_gt Exp(0.5 deg, 0.02 m) with ell = 0.3."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(batch):
        p = stereo_pair(seed=seed * 100 + b, n=n, semantic=False)
        r2 = np.random.default_rng(100000 + b)
        u = r2.normal(size=(n, 32)); u /= np.linalg.norm(u, axis=1, keepdims=True)
        v = r2.normal(size=(p.z.shape[0], 32)); v /= np.linalg.norm(v, axis=1, keepdims=True)
        T_eval = p.T_gt @ random_motion(rng, 0.5, 0.02)
        out.append(Pair(f"learned{b}", p.x, u.astype(np.float32), p.z, v.astype(np.float32),
                        [lin_block(32)], p.T_gt, 0.3, align={}, T_eval=T_eval))
    return out


def batched_pairs(seed=1004, batch=64, lo=2000, hi=60000, semantic=True):
    """Mixed stereo / RGB-D pairs, N and M ~ U[lo, hi] independently, per-pair
    motions of angle U[0,5] deg and translation U[0,0.3] m.  Rays are cast
    through random pixel subsets only (lazy rendering), so 64 pairs take
    seconds rather than minutes."""
    out = []
    for b in range(batch):
        r = np.random.default_rng(100000 + b + seed * 0)
        n = int(r.integers(lo, hi + 1))
        m = int(r.integers(lo, hi + 1))
        mot = random_motion(r, r.uniform(0.0, 5.0), r.uniform(0.0, 0.3))
        if b % 2 == 0:
            p = stereo_pair(seed=200000 + b, n=n, m=m, motion=mot, semantic=semantic, lazy=True)
        else:
            p = rgbd_pair(seed=200000 + b, n=n, m=m, motion=mot, lazy=True)
            if semantic:
                # give the RGB-D pair the same 5 + 19 feature layout
                s1 = r.dirichlet(np.full(19, 0.3), size=n).astype(np.float32)
                s2 = r.dirichlet(np.full(19, 0.3), size=m).astype(np.float32)
                p.u = np.concatenate([p.u, s1], axis=1)
                p.v = np.concatenate([p.v, s2], axis=1)
                p.spec = [se_block(5, 0.2), lin_block(19)]
        p.name = f"batch{b}_{'stereo' if b % 2 == 0 else 'rgbd'}"
        out.append(p)
    return out


def random_pair(seed, n, m, spec, extent=1.0, noise=0.05, angle_deg=3.0, trans=0.05):
    """Small unstructured pair for parity tests: X uniform in a cube of side
    2*extent, Z a noisy moved copy of a subset/extension of X."""
    rng = np.random.default_rng(seed)
    D = sum(b["dim"] for b in spec)
    x = rng.uniform(-extent, extent, (n, 3))
    T_gt = random_motion(rng, angle_deg, trans)
    base = x[rng.integers(0, n, m)] if m else np.zeros((0, 3))
    z = _apply(_inv(T_gt), base) + rng.normal(0.0, noise, base.shape)
    u = rng.uniform(0.0, 1.0, (n, D))
    v = rng.uniform(0.0, 1.0, (m, D))
    for b, off in zip(spec, np.cumsum([0] + [b["dim"] for b in spec])[:-1]):
        if b["kind"] == "lin":
            u[:, off:off + b["dim"]] = rng.dirichlet(np.ones(b["dim"]), size=n)
            v[:, off:off + b["dim"]] = rng.dirichlet(np.ones(b["dim"]), size=m)
    return Pair(f"random{seed}", x.astype(np.float32), u.astype(np.float32),
                z.astype(np.float32), v.astype(np.float32), list(spec), T_gt, 0.1)
