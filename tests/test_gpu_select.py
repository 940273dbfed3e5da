"""GPU parity of point selection (FAST 9-of-16 segment test, automatic
threshold, raster-order back-projection; Sec. IV's performance
considerations) against the oracle, through the C ABI: scores, threshold,
count and selected pixels bit for bit, points and features exactly."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import pose_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _check(cvo, gray, depth, feat, cam, cap):
    print(f"select {gray.shape} D={0 if feat is None else feat.shape[-1]} cap={cap}", flush=True)
    xyz, fo, t, sc = cvo.cvo_select_points(_dev(gray), _dev(depth), None if feat is None else _dev(feat), cam,
                                           cap, scores=True)
    oxyz, of, ot, oidx, osc = oracle.select_points(gray, depth, feat, cam, cap)
    np.testing.assert_array_equal(sc.cpu().numpy().astype(np.int32), osc)
    assert t == ot and xyz.shape[0] == oxyz.shape[0]
    np.testing.assert_array_equal(xyz.cpu().numpy(), oxyz)
    if feat is not None:
        np.testing.assert_array_equal(fo.cpu().numpy(), of)
    return xyz, fo, t


def test_select_full_frame_matches_oracle(cvo):
    s = synth.stereo_images(frames=1)
    fr = s.frames[0]
    xyz, fo, t = _check(cvo, fr.gray, fr.depth, fr.feat, s.camera, 15000)
    print("threshold", t, "points", xyz.shape[0])
    assert 3000 <= xyz.shape[0] <= 15000


@pytest.mark.parametrize("shape,cap", [((7, 7), 5), ((6, 40), 10), ((13, 70), 1), ((37, 131), 50),
                                       ((64, 256), 0), ((101, 67), 100000)])
def test_select_ragged_and_small_images(cvo, shape, cap):
    """Tiles with ragged right and bottom edges, images too small for an
    interior pixel, caps of 0 and 1, grey levels with exact ties, and depth
    values that are NaN, infinite, zero or outside the range."""
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    gray = rng.choice(np.array([0, 20, 21, 100, 180, 181, 255], np.uint8), size=shape)
    depth = rng.uniform(0.5, 12.0, size=shape).astype(np.float32)
    bad = rng.random(shape)
    depth[bad < 0.05] = np.nan
    depth[(bad >= 0.05) & (bad < 0.08)] = np.inf
    depth[(bad >= 0.08) & (bad < 0.12)] = 0.0
    feat = rng.random(shape + (7,)).astype(np.float32)
    cam = dict(fx=60.0, fy=58.5, cx=shape[1] / 2 - 0.5, cy=shape[0] / 2 + 0.25, depth_min=1.0, depth_max=10.0)
    _check(cvo, gray, depth, feat, cam, cap)
    _check(cvo, gray, depth, None, cam, cap)


def test_select_degenerate_inputs(cvo):
    cam = dict(fx=100.0, fy=100.0, cx=50.0, cy=40.0, depth_min=0.5, depth_max=5.0)
    flat = np.full((80, 100), 120, np.uint8)
    depth = np.full((80, 100), 2.0, np.float32)
    xyz, fo, t, sc = cvo.cvo_select_points(_dev(flat), _dev(depth), None, cam, 100, scores=True)
    assert xyz.shape[0] == 0 and t == 0 and (sc.cpu().numpy() == -1).all()
    rng = np.random.default_rng(5)
    noisy = rng.integers(0, 256, size=(80, 100)).astype(np.uint8)
    none = np.zeros((80, 100), np.float32)
    xyz, fo, t, sc = cvo.cvo_select_points(_dev(noisy), _dev(none), None, cam, 100)
    assert xyz.shape[0] == 0 and t == 0
    empty = np.zeros((0, 0), np.uint8)
    xyz, fo, t, sc = cvo.cvo_select_points(_dev(empty), _dev(np.zeros((0, 0), np.float32)), None, cam, 100)
    assert xyz.shape[0] == 0


def test_select_rejects_bad_arguments(cvo):
    lib = cvo.load_library()
    h = cvo.handle()
    g = _dev(np.zeros((10, 10), np.uint8))
    d = _dev(np.ones((10, 10), np.float32))
    out = torch.empty((8, 3), dtype=torch.float32, device="cuda:0")
    n, t = ctypes.c_int64(), ctypes.c_int32()
    good = cvo.cvo_camera(10.0, 10.0, 5.0, 5.0, 0.5, 2.0)
    args = lambda cam, cap, mp: (h, g.data_ptr(), d.data_ptr(), None, 10, 10, 0, ctypes.byref(cam), mp,
                                 out.data_ptr(), None, cap, None, ctypes.byref(n), ctypes.byref(t))
    assert lib.cvo_select_points(*args(good, 8, 8)) == 0
    assert lib.cvo_select_points(*args(good, 4, 8)) == cvo.CVO_ERR_INVALID_ARGUMENT
    bad = cvo.cvo_camera(10.0, 10.0, 5.0, 5.0, 0.0, 2.0)
    assert lib.cvo_select_points(*args(bad, 8, 8)) == cvo.CVO_ERR_INVALID_ARGUMENT
    bad = cvo.cvo_camera(-1.0, 10.0, 5.0, 5.0, 0.5, 2.0)
    assert lib.cvo_select_points(*args(bad, 8, 8)) == cvo.CVO_ERR_INVALID_ARGUMENT


def test_selected_frames_register(cvo):
    """The pipeline the selection serves: select 3k-15k points in each of two
    consecutive frames, then register them (ell 0.95 -> 0.1 from the
    identity); the estimate lands near the true relative pose."""
    s = synth.stereo_images(frames=2)
    clouds = []
    for fr in s.frames:
        xyz, fo, t = _check(cvo, fr.gray, fr.depth, fr.feat, s.camera, 15000)
        clouds.append((xyz, fo))
    (X, U), (Z, V) = clouds
    T, rep, _ = cvo.cvo_align(X, Z, U, V, s.spec, dict(ell_init=0.95, ell_min=0.1, max_iter=4000))
    ang, tr = pose_error(T, s.relative(0))
    print("selected", X.shape[0], Z.shape[0], rep, "error", np.degrees(ang), "deg", tr, "m")
    assert rep["status"] == cvo.CVO_CONVERGED
    assert np.degrees(ang) < 0.5 and tr < 0.1


def test_selected_frames_odometry(cvo):
    """The paper's pipeline on four image frames: select points in each frame,
    then frame-to-frame registration (the first pair from the identity with
    ell 0.95 -> 0.1, later pairs warm-started at 0.1); every relative pose
    lands near the truth and the chained trajectory drifts little."""
    s = synth.stereo_images(frames=4)
    sel = []
    for fr in s.frames:
        xyz, fo, t = _check(cvo, fr.gray, fr.depth, fr.feat, s.camera, 15000)
        assert 3000 <= xyz.shape[0] <= 15000
        sel.append((xyz, fo))
    Ts, reps = cvo.cvo_odometry(sel, s.spec, dict(ell_init=0.95, ell_min=0.1), dict(ell_init=0.1, ell_min=0.1))
    for k, T in enumerate(Ts):
        ang, tr = pose_error(T, s.relative(k))
        print(k, reps[k]["iterations"], np.degrees(ang), tr)
        assert reps[k]["status"] == cvo.CVO_CONVERGED
        assert np.degrees(ang) < 0.2 and tr < 0.03
    dt, dr = synth.trajectory_drift(s.poses, list(Ts))
    print("drift", dt, "%", dr, "deg/m")
    assert dt < 2.0 and dr < 0.1
