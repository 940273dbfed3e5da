"""MI355X (gfx950) continuous RKHS point-cloud registration (CVO, arXiv 2012.03683).

A thin ctypes binding over the C ABI of ``include/cvo.h`` (``libcvo_hip.so``,
built in-tree by ``paper_2012_03683_amd.build``).  The functions carry the C
names; they marshal arguments only -- every step of the computation runs in
the library's HIP kernels.  PyTorch provides the device memory and the
stream: clouds are CUDA (ROCm) float32 tensors, and each call enqueues on
``torch.cuda.current_stream()``.  There is no CPU fallback: without the
built library or a GPU every call raises.

Feature specs are lists of dicts ``{"kind": "se"|"lin", "dim": int,
"ell": float, "sigma": float}`` (see ``synth.se_block`` / ``synth.lin_block``).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcvo_hip.so")

CVO_OK, CVO_ERR_INVALID_ARGUMENT, CVO_ERR_OUT_OF_MEMORY, CVO_ERR_DEVICE, CVO_ERR_UNSUPPORTED = range(5)
CVO_SE, CVO_LIN = 0, 1
CVO_CONVERGED, CVO_MAX_ITER, CVO_NO_OVERLAP, CVO_STATIONARY = 1, 2, 3, 4
CVO_METRIC_KINETIC, CVO_METRIC_IDENTITY = 0, 1
CVO_ELL_ANNEAL, CVO_ELL_ADAPTIVE = 0, 1
CVO_CLUSTER_OCTREE, CVO_CLUSTER_CHUNKS = 0, 1
CVO_TRACE_LEN = 8
MAX_BLOCKS = 8

EXPORTS = ("cvo_create", "cvo_destroy", "cvo_set_stream", "cvo_last_error", "cvo_inner_product",
           "cvo_gradient", "cvo_evaluate", "cvo_evaluate_noalloc", "cvo_ell_objective", "cvo_metric", "cvo_cosine", "cvo_align", "cvo_align_replay",
           "cvo_inner_product_backward",
           "cvo_align_batched", "cvo_odometry", "cvo_select_points", "cvo_get_tuning", "cvo_set_tuning", "cvo_autotune",
           "cvo_set_profiling", "cvo_get_timing", "cvo_save_tuning", "cvo_load_tuning",
           "cvo_clear_tuning")


class CvoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cvo error {code}: {msg}")
        self.code = code


# ---------------------------------------------------------------- C structs
class cvo_cloud(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("feat", C.c_void_p), ("n", C.c_int64)]


class cvo_feature_spec(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("dim", C.c_int32 * MAX_BLOCKS), ("kind", C.c_int32 * MAX_BLOCKS),
                ("ell", C.c_double * MAX_BLOCKS), ("sigma", C.c_double * MAX_BLOCKS)]


class cvo_kernel_params(C.Structure):
    _fields_ = [("ell", C.c_double), ("sigma", C.c_double), ("kappa", C.c_double)]


class cvo_align_params(C.Structure):
    _fields_ = [("ell_init", C.c_double), ("ell_min", C.c_double), ("decay", C.c_double),
                ("ind_rel_tol", C.c_double), ("eps_rot", C.c_double), ("eps_trans", C.c_double),
                ("step_lambda", C.c_double), ("sigma", C.c_double), ("kappa", C.c_double),
                ("max_iter", C.c_int64), ("fixed_iters", C.c_int32), ("metric", C.c_int32),
                ("ell_mode", C.c_int32), ("reserved", C.c_int32)]


class cvo_align_report(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("final_ell", C.c_double), ("F", C.c_double),
                ("i_theta", C.c_double), ("n_pairs", C.c_int64), ("status", C.c_int32),
                ("reserved", C.c_int32), ("total_pairs", C.c_int64)]


class cvo_eval(C.Structure):
    _fields_ = [("F", C.c_double), ("grad", C.c_double * 6), ("curv", C.c_double), ("dF_dell", C.c_double),
                ("r_max", C.c_double), ("i_theta", C.c_double), ("n_pairs", C.c_int64)]


class cvo_tuning(C.Structure):
    _fields_ = [("cluster_max", C.c_int32), ("cell_factor", C.c_double), ("cluster_factor", C.c_double),
                ("rebuild_ratio", C.c_double), ("unroll", C.c_int32), ("piece_work", C.c_int32),
                ("cluster_rule", C.c_int32), ("adaptive", C.c_int32)]


class cvo_camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("depth_min", C.c_double), ("depth_max", C.c_double)]


class cvo_timing(C.Structure):
    _fields_ = [("pair_launches", C.c_int64), ("pair_ms", C.c_double), ("pair_count", C.c_int64),
                ("evaluations", C.c_int64), ("graph_launches", C.c_int64), ("graph_captures", C.c_int64),
                ("view_builds", C.c_int64), ("host_waits", C.c_int64), ("tuned_view_shapes", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcvo_hip.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2012_03683_amd.build`")
    lib = C.CDLL(path)
    P = C.POINTER
    H = C.c_void_p
    lib.cvo_create.argtypes = [P(H), C.c_int, C.c_void_p]
    lib.cvo_destroy.argtypes = [H]
    lib.cvo_destroy.restype = None
    lib.cvo_set_stream.argtypes = [H, C.c_void_p]
    lib.cvo_last_error.argtypes = [H]
    lib.cvo_last_error.restype = C.c_char_p
    common = [H, P(cvo_cloud), P(cvo_cloud), P(cvo_feature_spec), P(cvo_kernel_params), C.c_void_p]
    lib.cvo_inner_product.argtypes = common + [P(C.c_double), P(C.c_int64)]
    lib.cvo_gradient.argtypes = common + [P(C.c_double), C.c_void_p, P(C.c_int64)]
    lib.cvo_evaluate.argtypes = common + [P(cvo_eval)]
    lib.cvo_evaluate_noalloc.argtypes = common + [P(cvo_eval)]
    lib.cvo_ell_objective.argtypes = common + [C.c_void_p]
    lib.cvo_metric.argtypes = common + [P(C.c_double)]
    lib.cvo_cosine.argtypes = common + [P(C.c_double), C.c_void_p]
    lib.cvo_align.argtypes = [H, P(cvo_cloud), P(cvo_cloud), P(cvo_feature_spec), P(cvo_align_params),
                              C.c_void_p, C.c_void_p, P(cvo_align_report), C.c_void_p]
    lib.cvo_align_replay.argtypes = [H, P(cvo_cloud), P(cvo_cloud), P(cvo_feature_spec), P(cvo_align_params),
                                     C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, P(cvo_align_report),
                                     C.c_void_p]
    lib.cvo_inner_product_backward.argtypes = common + [C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                                        C.c_void_p, P(C.c_double)]
    lib.cvo_align_batched.argtypes = [H, C.c_int32, P(cvo_cloud), P(cvo_cloud), P(cvo_feature_spec),
                                      P(cvo_align_params), C.c_int32, C.c_void_p, C.c_void_p,
                                      P(cvo_align_report)]
    lib.cvo_odometry.argtypes = [H, C.c_int32, P(cvo_cloud), P(cvo_feature_spec), P(cvo_align_params),
                                 P(cvo_align_params), C.c_void_p, P(cvo_align_report)]
    lib.cvo_select_points.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                      P(cvo_camera), C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                      P(C.c_int64), P(C.c_int32)]
    lib.cvo_get_tuning.argtypes = [H, P(cvo_tuning)]
    lib.cvo_set_tuning.argtypes = [H, P(cvo_tuning)]
    lib.cvo_autotune.argtypes = common + [P(cvo_tuning)]
    lib.cvo_save_tuning.argtypes = [H, C.c_char_p]
    lib.cvo_load_tuning.argtypes = [H, C.c_char_p]
    lib.cvo_clear_tuning.argtypes = [H]
    lib.cvo_set_profiling.argtypes = [H, C.c_int32]
    lib.cvo_get_timing.argtypes = [H, P(cvo_timing)]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name not in ("cvo_destroy", "cvo_last_error"):
            f.restype = C.c_int
    _lib = lib
    return lib


# ---------------------------------------------------------------- handles
_handles = {}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the CVO library runs on MI355X (gfx950) only")
    return torch


def handle(device=None):
    """The per-device library handle, bound to torch's current stream."""
    torch = _torch()
    lib = load_library()
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _handles.get(dev)
    if h is None:
        hh = C.c_void_p()
        rc = lib.cvo_create(C.byref(hh), dev, None)
        if rc != CVO_OK:
            raise CvoError(rc, f"cvo_create failed on device {dev}")
        h = hh
        _handles[dev] = h
    lib.cvo_set_stream(h, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    return h


def _check(rc, h):
    if rc != CVO_OK:
        raise CvoError(rc, load_library().cvo_last_error(h).decode())


def _spec(spec):
    s = cvo_feature_spec()
    spec = list(spec or [])
    if len(spec) > MAX_BLOCKS:
        raise ValueError("at most 8 feature blocks")
    s.nblocks = len(spec)
    for b, blk in enumerate(spec):
        s.dim[b] = int(blk["dim"])
        s.kind[b] = CVO_SE if blk["kind"] == "se" else CVO_LIN
        s.ell[b] = float(blk.get("ell", 1.0))
        s.sigma[b] = float(blk.get("sigma", 1.0))
    return s


def _dev_f32(t, cols, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.device.type != "cuda":
        raise ValueError(f"{name} is on {t.device}; the CVO library has no CPU path")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"{name} must have shape (n, {cols})")
    return t.contiguous()


def _cloud(xyz, feat, D, name):
    xyz = _dev_f32(xyz, 3, name)
    keep = [xyz]
    fptr = None
    if D:
        if feat is None:
            raise ValueError(f"{name}: the spec has {D} feature columns but no features were given")
        feat = _dev_f32(feat, D, name + " features")
        if feat.shape[0] != xyz.shape[0]:
            raise ValueError(f"{name}: feature rows differ from point count")
        keep.append(feat)
        fptr = feat.data_ptr()
    return cvo_cloud(xyz.data_ptr(), fptr, xyz.shape[0]), keep


def _pose(T):
    T = np.asarray(T, dtype=np.float64)
    if T.shape == (4, 4):
        T = T[:3]
    if T.shape != (3, 4):
        raise ValueError("pose must be 4x4 or 3x4")
    return np.ascontiguousarray(T).reshape(12).copy()


def _dim(spec):
    return int(sum(int(b["dim"]) for b in (spec or [])))


def _prep(X, Z, U, V, spec):
    D = _dim(spec)
    cx, kx = _cloud(X, U, D, "X")
    cz, kz = _cloud(Z, V, D, "Z")
    return cx, cz, kx + kz, _spec(spec)


# ---------------------------------------------------------------- the C calls
def cvo_inner_product(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    """F of eq. (7) and the exact pair count |P| at pose T."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    F = C.c_double()
    n = C.c_int64()
    _check(load_library().cvo_inner_product(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp),
                                            Tp.ctypes.data, C.byref(F), C.byref(n)), h)
    del keep
    return F.value, int(n.value)


def cvo_gradient(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    """F and its se(3) gradient (omega, v) at T."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    F = C.c_double()
    g = np.zeros(6)
    n = C.c_int64()
    _check(load_library().cvo_gradient(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data,
                                       C.byref(F), g.ctypes.data, C.byref(n)), h)
    del keep
    return F.value, g, int(n.value)


def cvo_evaluate(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0, noalloc=False):
    """All outputs of one pair pass as a dict.  noalloc=True calls
    cvo_evaluate_noalloc (scratch from the library's fixed device array)."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    out = cvo_eval()
    fn = load_library().cvo_evaluate_noalloc if noalloc else load_library().cvo_evaluate
    _check(fn(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data, C.byref(out)), h)
    del keep
    return {"F": out.F, "grad": np.array(out.grad[:]), "curv": out.curv, "dF_dell": out.dF_dell,
            "r_max": out.r_max, "i_theta": out.i_theta, "n_pairs": int(out.n_pairs)}


def cvo_cosine(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    """Cosine of the angle between f_X and the moved f_Z (eq. (9)); returns
    (cos_theta, F(X,Z;T), F(X,X;I), F(Z,Z;I))."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    v = C.c_double()
    sums = (C.c_double * 3)()
    _check(load_library().cvo_cosine(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data,
                                     C.byref(v), sums), h)
    del keep
    return v.value, sums[0], sums[1], sums[2]


def cvo_metric(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    """Alignment indicator i_theta of eq. (10)."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    v = C.c_double()
    _check(load_library().cvo_metric(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data,
                                     C.byref(v)), h)
    del keep
    return v.value


DEFAULT_ALIGN = dict(ell_init=0.1, ell_min=0.1, decay=0.98, ind_rel_tol=1e-3, eps_rot=1e-6, eps_trans=1e-6,
                     step_lambda=1.0, sigma=1.0, kappa=3.0, max_iter=4000, fixed_iters=False,
                     metric=CVO_METRIC_KINETIC, ell_mode=CVO_ELL_ANNEAL)


def _align_params(params):
    p = dict(DEFAULT_ALIGN)
    p.update(params or {})
    return cvo_align_params(p["ell_init"], p["ell_min"], p["decay"], p["ind_rel_tol"], p["eps_rot"],
                            p["eps_trans"], p["step_lambda"], p["sigma"], p["kappa"], int(p["max_iter"]),
                            int(bool(p["fixed_iters"])), int(p["metric"]), int(p["ell_mode"]), 0), p


def _report(r):
    return {"iterations": int(r.iterations), "final_ell": r.final_ell, "F": r.F, "i_theta": r.i_theta,
            "n_pairs": int(r.n_pairs), "status": int(r.status), "total_pairs": int(r.total_pairs)}


def cvo_align(X, Z, U=None, V=None, spec=None, params=None, T_init=None, trace=False):
    """Problem 1 ascent with annealing; returns (T 4x4, report, trace or None)."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    ap, p = _align_params(params)
    T0 = _pose(np.eye(4) if T_init is None else T_init)
    Tout = np.zeros(12)
    rep = cvo_align_report()
    tr = np.zeros((int(p["max_iter"]), CVO_TRACE_LEN)) if trace else None
    _check(load_library().cvo_align(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(ap), T0.ctypes.data,
                                    Tout.ctypes.data, C.byref(rep), tr.ctypes.data if trace else None), h)
    del keep
    T = np.eye(4)
    T[:3] = Tout.reshape(3, 4)
    r = _report(rep)
    return T, r, (tr[:r["iterations"]].copy() if trace else None)


def cvo_align_batched(pairs, spec=None, params=None, T_init=None):
    """Register B pairs [(X, Z, U, V), ...] in one device-resident loop.
    params: dict or list of B dicts; T_init: None or array (B, 4, 4)."""
    h = handle()
    B = len(pairs)
    D = _dim(spec)
    xs = (cvo_cloud * B)()
    zs = (cvo_cloud * B)()
    keep = []
    for b, (X, Z, U, V) in enumerate(pairs):
        xs[b], k1 = _cloud(X, U, D, f"X[{b}]")
        zs[b], k2 = _cloud(Z, V, D, f"Z[{b}]")
        keep += k1 + k2
    plist = params if isinstance(params, (list, tuple)) else [params]
    aps = (cvo_align_params * len(plist))(*[_align_params(p)[0] for p in plist])
    T0 = np.zeros((B, 12))
    for b in range(B):
        T0[b] = _pose(np.eye(4) if T_init is None else T_init[b])
    Tout = np.zeros((B, 12))
    reps = (cvo_align_report * B)()
    sp = _spec(spec)
    _check(load_library().cvo_align_batched(h, B, xs, zs, C.byref(sp), aps, len(plist), T0.ctypes.data,
                                            Tout.ctypes.data, reps), h)
    del keep
    Ts = np.tile(np.eye(4), (B, 1, 1))
    Ts[:, :3, :] = Tout.reshape(B, 3, 4)
    return Ts, [_report(r) for r in reps]


def cvo_align_replay(X, Z, U=None, V=None, spec=None, ell_sched=(), params=None, T_init=None, trace=False):
    """cvo_align with the lengthscale of iteration i fixed to ell_sched[i]
    (no annealing decisions, exactly len(ell_sched) iterations); returns
    (T 4x4, report, trace or None)."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    ap, p = _align_params(params)
    sched = np.ascontiguousarray(np.asarray(ell_sched, dtype=np.float64).reshape(-1))
    T0 = _pose(np.eye(4) if T_init is None else T_init)
    Tout = np.zeros(12)
    rep = cvo_align_report()
    tr = np.zeros((max(sched.size, 1), CVO_TRACE_LEN)) if trace else None
    _check(load_library().cvo_align_replay(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(ap), T0.ctypes.data,
                                           sched.ctypes.data if sched.size else None, sched.size, Tout.ctypes.data,
                                           C.byref(rep), tr.ctypes.data if trace else None), h)
    del keep
    T = np.eye(4)
    T[:3] = Tout.reshape(3, 4)
    r = _report(rep)
    return T, r, (tr[:r["iterations"]].copy() if trace else None)


def cvo_odometry(frames, spec=None, first=None, rest=None):
    """Frame-to-frame registration of a sequence [(xyz, feat), ...] of device
    tensors: pair k registers frame k + 1 to frame k, pair 0 from the identity
    with `first`, later pairs from the previous estimate with `rest`.
    Returns (relative poses (F-1, 4, 4), reports)."""
    h = handle()
    F = len(frames)
    D = _dim(spec)
    fs = (cvo_cloud * F)()
    keep = []
    for k, (X, U) in enumerate(frames):
        fs[k], kk = _cloud(X, U, D, f"frame[{k}]")
        keep += kk
    a0, _ = _align_params(first)
    a1, _ = _align_params(rest)
    Tout = np.zeros((max(F - 1, 0), 12))
    reps = (cvo_align_report * max(F - 1, 1))()
    sp = _spec(spec)
    _check(load_library().cvo_odometry(h, F, fs, C.byref(sp), C.byref(a0), C.byref(a1), Tout.ctypes.data,
                                       reps), h)
    del keep
    Ts = np.tile(np.eye(4), (F - 1, 1, 1))
    Ts[:, :3, :] = Tout.reshape(F - 1, 3, 4)
    return Ts, [_report(r) for r in reps]


def _dev_image(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.device.type != "cuda":
        raise ValueError(f"{name} is on {t.device}; the CVO library has no CPU path")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}")
    return t.contiguous()


def cvo_select_points(gray, depth, feat=None, camera=None, max_points=15000, scores=False):
    """Point selection on device images (FAST 9-of-16, threshold chosen so at
    most max_points pixels with depth are kept).  gray (H, W) uint8, depth
    (H, W) float32, feat (H, W, D) float32 or None, camera a dict of fx, fy,
    cx, cy, depth_min, depth_max.  Returns (xyz (n, 3), feat (n, D),
    threshold, scores (H, W) int16 or None)."""
    torch = _torch()
    h = handle()
    H, W = gray.shape
    gray = _dev_image(gray, torch.uint8, (H, W), "gray")
    depth = _dev_image(depth, torch.float32, (H, W), "depth")
    D = 0 if feat is None else int(feat.shape[-1])
    if D:
        feat = _dev_image(feat, torch.float32, (H, W, D), "feat")
    cam = cvo_camera(camera["fx"], camera["fy"], camera["cx"], camera["cy"], camera["depth_min"],
                     camera["depth_max"])
    cap = int(max_points)
    xyz = torch.empty((cap, 3), dtype=torch.float32, device=gray.device)
    fo = torch.empty((cap, D), dtype=torch.float32, device=gray.device)
    sc = torch.empty((H, W), dtype=torch.int16, device=gray.device) if scores else None
    n = C.c_int64()
    t = C.c_int32()
    ptr = (lambda x: x.data_ptr() if (x is not None and x.numel()) else None)
    _check(load_library().cvo_select_points(h, ptr(gray), ptr(depth), ptr(feat) if D else None, W, H, D,
                                            C.byref(cam), cap, ptr(xyz), ptr(fo), cap, ptr(sc), C.byref(n),
                                            C.byref(t)), h)
    k = int(n.value)
    return xyz[:k], fo[:k], int(t.value), sc


def cvo_inner_product_backward(X, Z, T, ell, gF=1.0, U=None, V=None, spec=None, sigma=1.0, kappa=3.0,
                               need=("x", "z", "u", "v", "ell")):
    """Derivatives of gF * F w.r.t. positions, features and ell (frozen pair set)."""
    torch = _torch()
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    D = _dim(spec)
    dX = torch.empty((X.shape[0], 3), device=X.device, dtype=torch.float32) if "x" in need else None
    dZ = torch.empty((Z.shape[0], 3), device=X.device, dtype=torch.float32) if "z" in need else None
    dU = torch.empty((X.shape[0], D), device=X.device, dtype=torch.float32) if ("u" in need and D) else None
    dV = torch.empty((Z.shape[0], D), device=X.device, dtype=torch.float32) if ("v" in need and D) else None
    dl = C.c_double()
    ptr = (lambda t: t.data_ptr() if t is not None else None)
    _check(load_library().cvo_inner_product_backward(
        h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data, float(gF), ptr(dX), ptr(dZ),
        ptr(dU), ptr(dV), C.byref(dl) if "ell" in need else None), h)
    del keep
    return {"dX": dX, "dZ": dZ, "dU": dU, "dV": dV, "dell": dl.value if "ell" in need else None}


def cvo_ell_objective(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    """Lengthscale objective of the adaptive mode: J = sum_{W_j > 0} log W_j -
    3 |Z+| log ell on the pair set frozen at (T, ell), dJ/dell, its maximiser
    ell_ml and |Z+| (cvo_ell_objective)."""
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    out = np.zeros(4)
    _check(load_library().cvo_ell_objective(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp),
                                            Tp.ctypes.data, out.ctypes.data), h)
    del keep
    return {"J": out[0], "dJ_dell": out[1], "ell_ml": out[2], "n_plus": int(out[3])}


def cvo_evaluate_noalloc(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    """cvo_evaluate through the allocation-free entry point."""
    return cvo_evaluate(X, Z, T, ell, U, V, spec, sigma, kappa, noalloc=True)


def cvo_get_tuning():
    h = handle()
    t = cvo_tuning()
    _check(load_library().cvo_get_tuning(h, C.byref(t)), h)
    return {k: getattr(t, k) for k, _ in cvo_tuning._fields_ if k != "reserved"}


def cvo_set_tuning(**kw):
    h = handle()
    t = cvo_tuning()
    _check(load_library().cvo_get_tuning(h, C.byref(t)), h)
    for k, v in kw.items():
        setattr(t, k, v)
    _check(load_library().cvo_set_tuning(h, C.byref(t)), h)


def cvo_autotune(X, Z, T, ell, U=None, V=None, spec=None, sigma=1.0, kappa=3.0):
    h = handle()
    cx, cz, keep, sp = _prep(X, Z, U, V, spec)
    kp = cvo_kernel_params(ell, sigma, kappa)
    Tp = _pose(T)
    t = cvo_tuning()
    _check(load_library().cvo_autotune(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data,
                                       C.byref(t)), h)
    del keep
    return {k: getattr(t, k) for k, _ in cvo_tuning._fields_ if k != "reserved"}


def cvo_save_tuning(path):
    """Write the autotuner's class table and one-shot cache to a text file."""
    h = handle()
    _check(load_library().cvo_save_tuning(h, os.fsencode(path)), h)


def cvo_load_tuning(path):
    """Merge a tuning file written by cvo_save_tuning into the handle."""
    h = handle()
    _check(load_library().cvo_load_tuning(h, os.fsencode(path)), h)


def cvo_clear_tuning():
    """Forget the autotuner's class table and one-shot cache."""
    h = handle()
    _check(load_library().cvo_clear_tuning(h), h)


def cvo_set_profiling(enable=True):
    h = handle()
    _check(load_library().cvo_set_profiling(h, int(bool(enable))), h)


def cvo_get_timing():
    h = handle()
    t = cvo_timing()
    _check(load_library().cvo_get_timing(h, C.byref(t)), h)
    return {k: (getattr(t, k) if k == "pair_ms" else int(getattr(t, k))) for k, _ in cvo_timing._fields_}


# ---------------------------------------------------------------- autograd
def _make_autograd():
    import torch

    class CvoInnerProduct(torch.autograd.Function):
        """F = <f_X, f_{T Z}> (eq. (7)) with a hand-written backward giving
        dF/dX, dF/dZ, dF/dU, dF/dV and dF/dell on the frozen pair set.
        apply(X, Z, U, V, T(4x4 numpy or tensor, not differentiated), ell(float or
        0-dim tensor), spec, sigma, kappa) -> 0-dim float64 tensor."""

        @staticmethod
        def forward(ctx, X, Z, U, V, T, ell, spec, sigma=1.0, kappa=3.0):
            ell_f = float(ell)
            Tn = T.detach().cpu().numpy() if isinstance(T, torch.Tensor) else np.asarray(T)
            F, _ = cvo_inner_product(X.detach(), Z.detach(), Tn, ell_f,
                                     U.detach() if U is not None else None,
                                     V.detach() if V is not None else None, spec, sigma, kappa)
            ctx.save_for_backward(X, Z, *([U, V] if U is not None else []))
            ctx.meta = (Tn, ell_f, spec, sigma, kappa, U is not None, isinstance(ell, torch.Tensor))
            return torch.tensor(F, dtype=torch.float64, device=X.device)

        @staticmethod
        def backward(ctx, gF):
            Tn, ell_f, spec, sigma, kappa, has_feat, ell_is_t = ctx.meta
            saved = ctx.saved_tensors
            X, Z = saved[0].detach(), saved[1].detach()
            U, V = (saved[2].detach(), saved[3].detach()) if has_feat else (None, None)
            g = float(gF.item())
            r = cvo_inner_product_backward(X, Z, Tn, ell_f, g, U, V, spec, sigma, kappa)
            dell = torch.tensor(r["dell"], dtype=torch.float64, device=X.device) if ell_is_t else None
            return r["dX"], r["dZ"], r["dU"], r["dV"], None, dell, None, None, None

    return CvoInnerProduct


def __getattr__(name):
    if name == "CvoInnerProduct":
        f = _make_autograd()
        globals()["CvoInnerProduct"] = f
        return f
    raise AttributeError(name)
