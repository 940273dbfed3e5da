"""FP64 CPU oracle for the CVO hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package imports nothing from it.

The registration arithmetic lives in ``cvo_oracle.c`` (plain C, every
operation a rounded IEEE double, no FMA); this module only marshals numpy
arrays through ctypes.  Point selection (``select.py``) is plain integer
numpy from the FAST definition.
Feature specs are plain lists of dicts ``{"kind": "se"|"lin", "dim": int,
"ell": float, "sigma": float}``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .select import fast_scores, select_points, select_threshold, valid_depth  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcvo_oracle.so")
_SRC = os.path.join(_HERE, "cvo_oracle.c")

SE, LIN = 0, 1
CONVERGED, MAX_ITER, NO_OVERLAP, STATIONARY = 1, 2, 3, 4
METRIC_KINETIC, METRIC_IDENTITY = 0, 1
ELL_ANNEAL, ELL_ADAPTIVE = 0, 1
EVAL_LEN, TRACE_LEN, REPORT_LEN = 18, 8, 6
MAX_BLOCKS = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Cloud(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("feat", C.c_void_p), ("n", C.c_int64)]


class _Spec(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("dim", C.c_int32 * MAX_BLOCKS),
                ("kind", C.c_int32 * MAX_BLOCKS), ("ell", C.c_double * MAX_BLOCKS),
                ("sigma", C.c_double * MAX_BLOCKS)]


class _AlignParams(C.Structure):
    _fields_ = [("ell_init", C.c_double), ("ell_min", C.c_double), ("decay", C.c_double),
                ("ind_rel_tol", C.c_double), ("eps_rot", C.c_double), ("eps_trans", C.c_double),
                ("step_lambda", C.c_double), ("sigma", C.c_double), ("kappa", C.c_double),
                ("max_iter", C.c_int64), ("fixed_iters", C.c_int32), ("metric", C.c_int32),
                ("ell_mode", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = C.CDLL(_SO)
        P = C.POINTER
        lib.oracle_evaluate.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                        C.c_double, C.c_void_p, C.c_void_p, P(C.c_int64)]
        lib.oracle_target_moments.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                              C.c_double, C.c_void_p, C.c_void_p, C.c_int64,
                                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_evaluate_dir.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                            C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, P(C.c_int64)]
        lib.oracle_ell_objective.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                             C.c_double, C.c_void_p, C.c_void_p]
        lib.oracle_metric_tensor.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        lib.oracle_metric_tensor.restype = None
        lib.oracle_solve6.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_exp_se3.argtypes = [C.c_void_p, C.c_void_p]
        lib.oracle_exp_se3.restype = None
        lib.oracle_transform.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        lib.oracle_transform.restype = None
        lib.oracle_align.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), P(_AlignParams), C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_backward.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                        C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        lib.oracle_source_grad.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                           C.c_double, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.c_void_p]
        lib.oracle_target_grad.argtypes = [P(_Cloud), P(_Cloud), P(_Spec), C.c_double, C.c_double,
                                           C.c_double, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.c_void_p]
        lib.oracle_num_threads.restype = C.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _f32(a, cols):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.size == 0:
        return a.reshape(0, cols)
    return a.reshape(-1, cols)


def _pose(T):
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64)[:3, :4])
    return T.reshape(12).copy()


def _spec(spec):
    s = _Spec()
    spec = list(spec or [])
    if len(spec) > MAX_BLOCKS:
        raise ValueError("too many feature blocks")
    s.nblocks = len(spec)
    for b, blk in enumerate(spec):
        s.dim[b] = int(blk["dim"])
        s.kind[b] = SE if blk["kind"] == "se" else LIN
        s.ell[b] = float(blk.get("ell", 1.0))
        s.sigma[b] = float(blk.get("sigma", 1.0))
    return s


class _Pair:
    """Keeps the numpy buffers alive while ctypes holds raw pointers."""

    def __init__(self, x, u, z, v, spec):
        D = sum(int(b["dim"]) for b in (spec or []))
        self.D = D
        self.x = _f32(x, 3)
        self.z = _f32(z, 3)
        self.u = _f32(u, D) if D else None
        self.v = _f32(v, D) if D else None
        if D and (self.u.shape[0] != self.x.shape[0] or self.v.shape[0] != self.z.shape[0]):
            raise ValueError("feature rows must match point counts")
        self.X = _Cloud(self.x.ctypes.data, self.u.ctypes.data if D else None, self.x.shape[0])
        self.Z = _Cloud(self.z.ctypes.data, self.v.ctypes.data if D else None, self.z.shape[0])
        self.S = _spec(spec)


def evaluate(x, u, z, v, spec, ell, T=None, sigma=1.0, kappa=3.0, direction=None):
    """F, gradient (omega, v), curvature along the gradient (or along
    `direction`), dF/dell, |P| (eq. (7))."""
    p = _Pair(x, u, z, v, spec)
    T = _pose(np.eye(4) if T is None else T)
    out = np.zeros(EVAL_LEN, np.float64)
    n = C.c_int64(0)
    dptr = None
    if direction is not None:
        dvec = np.ascontiguousarray(np.asarray(direction, np.float64).reshape(6))
        dptr = dvec.ctypes.data
    rc = _load().oracle_evaluate_dir(C.byref(p.X), C.byref(p.Z), C.byref(p.S), ell, sigma, kappa,
                                     T.ctypes.data, dptr, out.ctypes.data, C.byref(n))
    if rc:
        raise ValueError(f"oracle_evaluate failed ({rc})")
    return {"F": out[0], "grad": out[1:7].copy(), "phi2": out[7], "dF_dell": out[8],
            "absF": out[9], "absgrad": out[10:16].copy(), "r_max": out[16],
            "i_theta": out[17], "n_pairs": int(n.value)}


def cosine(x, u, z, v, spec, ell, T=None, sigma=1.0, kappa=3.0):
    """Cosine of the angle between f_X and the moved f_Z (eq. (9), Sec. III-C):
    <f_X, h.f_Z> / (||f_X|| ||f_Z||), the squared norms being the self inner
    products F(X, X; I) and F(Z, Z; I) with the same kernels and cutoff.
    Returns (cos_theta, F_XZ, F_XX, F_ZZ); cos_theta is 0 when a squared norm
    is not positive."""
    fxz = evaluate(x, u, z, v, spec, ell, T, sigma, kappa)["F"]
    fxx = evaluate(x, u, x, u, spec, ell, None, sigma, kappa)["F"]
    fzz = evaluate(z, v, z, v, spec, ell, None, sigma, kappa)["F"]
    c = fxz / (np.sqrt(fxx) * np.sqrt(fzz)) if fxx > 0 and fzz > 0 else 0.0
    return c, fxz, fxx, fzz


def target_moments(x, u, z, v, spec, ell, idx, T=None, sigma=1.0, kappa=3.0):
    """Per-target W_j, D_j, S_j (upper triangle), n_j for targets j in idx."""
    p = _Pair(x, u, z, v, spec)
    T = _pose(np.eye(4) if T is None else T)
    idx = np.ascontiguousarray(np.asarray(idx, np.int64))
    k = idx.shape[0]
    W = np.zeros(k); Dm = np.zeros((k, 3)); S = np.zeros((k, 6)); cnt = np.zeros(k, np.int64)
    rc = _load().oracle_target_moments(C.byref(p.X), C.byref(p.Z), C.byref(p.S), ell, sigma, kappa,
                                       T.ctypes.data, idx.ctypes.data, k, W.ctypes.data,
                                       Dm.ctypes.data, S.ctypes.data, cnt.ctypes.data)
    if rc:
        raise ValueError(f"oracle_target_moments failed ({rc})")
    return W, Dm, S, cnt


def exp_se3(xi):
    """SE(3) exponential of xi = (omega, v) as a 4x4 matrix."""
    xi = np.ascontiguousarray(np.asarray(xi, np.float64).reshape(6))
    T = np.zeros(12)
    _load().oracle_exp_se3(xi.ctypes.data, T.ctypes.data)
    out = np.eye(4)
    out[:3, :4] = T.reshape(3, 4)
    return out


def transform(T, z):
    """Canonical z' = R z + t in FP64 (the operation order the pair predicate uses)."""
    z = _f32(z, 3)
    T = _pose(T)
    out = np.zeros((z.shape[0], 3))
    _load().oracle_transform(T.ctypes.data, z.ctypes.data, z.shape[0], out.ctypes.data)
    return out


DEFAULT_ALIGN = dict(ell_init=0.1, ell_min=0.1, decay=0.98, ind_rel_tol=1e-3, eps_rot=1e-6,
                     eps_trans=1e-6, step_lambda=1.0, sigma=1.0, kappa=3.0, max_iter=4000,
                     fixed_iters=False, metric=METRIC_KINETIC, ell_mode=ELL_ANNEAL)


def ell_objective(x, u, z, v, spec, ell, T=None, sigma=1.0, kappa=3.0):
    """The lengthscale objective of the adaptive mode (Sec. VI): J(T, ell) =
    sum_{W_j > 0} log W_j - 3 |Z+| log ell on the pair set frozen at (T, ell),
    its ell-derivative, the maximum-likelihood lengthscale
    sqrt(sum_j r_j / (3 |Z+|)) (r_j = target j's weighted mean squared
    residual) and |Z+|."""
    p = _Pair(x, u, z, v, spec)
    T = _pose(np.eye(4) if T is None else T)
    out = np.zeros(4)
    rc = _load().oracle_ell_objective(C.byref(p.X), C.byref(p.Z), C.byref(p.S), ell, sigma, kappa,
                                      T.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError(f"oracle_ell_objective failed ({rc})")
    return {"J": out[0], "dJ_dell": out[1], "ell_ml": out[2], "n_plus": int(out[3])}


def metric_tensor(T, z):
    """The kinetic-energy metric G of the moving cloud at pose T (6x6)."""
    z = _f32(z, 3)
    T = _pose(T)
    G = np.zeros(36)
    _load().oracle_metric_tensor(T.ctypes.data, z.ctypes.data, z.shape[0], G.ctypes.data)
    return G.reshape(6, 6)


def solve6(G, g):
    G = np.ascontiguousarray(np.asarray(G, np.float64).reshape(36))
    g = np.ascontiguousarray(np.asarray(g, np.float64).reshape(6))
    d = np.zeros(6)
    if _load().oracle_solve6(G.ctypes.data, g.ctypes.data, d.ctypes.data):
        raise ValueError("singular metric")
    return d


def align(x, u, z, v, spec, params=None, T_init=None, trace=True):
    """Problem 1 ascent with annealing; returns (T 4x4, report dict, trace array)."""
    p = _Pair(x, u, z, v, spec)
    prm = dict(DEFAULT_ALIGN)
    prm.update(params or {})
    ap = _AlignParams(prm["ell_init"], prm["ell_min"], prm["decay"], prm["ind_rel_tol"],
                      prm["eps_rot"], prm["eps_trans"], prm["step_lambda"], prm["sigma"],
                      prm["kappa"], int(prm["max_iter"]), int(bool(prm["fixed_iters"])),
                      int(prm["metric"]), int(prm["ell_mode"]), 0)
    T0 = _pose(np.eye(4) if T_init is None else T_init)
    Tout = np.zeros(12)
    rep = np.zeros(REPORT_LEN)
    tr = np.zeros((int(prm["max_iter"]), TRACE_LEN)) if trace else None
    rc = _load().oracle_align(C.byref(p.X), C.byref(p.Z), C.byref(p.S), C.byref(ap), T0.ctypes.data,
                              Tout.ctypes.data, rep.ctypes.data, tr.ctypes.data if trace else None)
    if rc:
        raise ValueError(f"oracle_align failed ({rc})")
    T = np.eye(4)
    T[:3, :4] = Tout.reshape(3, 4)
    it = int(rep[0])
    report = {"iterations": it, "final_ell": rep[1], "F": rep[2], "i_theta": rep[3],
              "n_pairs": int(rep[4]), "status": int(rep[5])}
    return T, report, (tr[:it].copy() if trace else None)


def odometry(frames, spec, first=None, rest=None):
    """Frame-to-frame registration (Sec. IV): pair k registers frame k + 1 to
    frame k; the first pair starts at the identity with `first`, every later
    one at the previous pair's estimate with `rest`.  frames = [(xyz, feat)];
    returns the relative poses (4x4, frame k + 1 into frame k) and reports."""
    T = np.eye(4)
    rel, reps = [], []
    for k in range(len(frames) - 1):
        (x, u), (z, v) = frames[k], frames[k + 1]
        T, rep, _ = align(x, u, z, v, spec, first if k == 0 else rest, T_init=T, trace=False)
        rel.append(T)
        reps.append(rep)
    return rel, reps


def backward(x, u, z, v, spec, ell, T=None, sigma=1.0, kappa=3.0):
    """dF/dx, dF/dz, dF/du, dF/dv, dF/dell on the frozen pair set."""
    p = _Pair(x, u, z, v, spec)
    T = _pose(np.eye(4) if T is None else T)
    N, M, D = p.x.shape[0], p.z.shape[0], p.D
    dx = np.zeros((N, 3)); dz = np.zeros((M, 3))
    du = np.zeros((N, D)); dv = np.zeros((M, D))
    dl = C.c_double(0.0)
    rc = _load().oracle_backward(C.byref(p.X), C.byref(p.Z), C.byref(p.S), ell, sigma, kappa,
                                 T.ctypes.data, dx.ctypes.data, dz.ctypes.data,
                                 du.ctypes.data if D else None, dv.ctypes.data if D else None,
                                 C.byref(dl))
    if rc:
        raise ValueError(f"oracle_backward failed ({rc})")
    return {"dx": dx, "dz": dz, "du": du, "dv": dv, "dell": dl.value}


def source_grad(x, u, z, v, spec, ell, idx, T=None, sigma=1.0, kappa=3.0):
    """dF/dx_i and dF/du_i for the sources i in idx only."""
    p = _Pair(x, u, z, v, spec)
    T = _pose(np.eye(4) if T is None else T)
    idx = np.ascontiguousarray(np.asarray(idx, np.int64))
    k = idx.shape[0]
    dx = np.zeros((k, 3)); du = np.zeros((k, max(p.D, 1)))
    rc = _load().oracle_source_grad(C.byref(p.X), C.byref(p.Z), C.byref(p.S), ell, sigma, kappa,
                                    T.ctypes.data, idx.ctypes.data, k, dx.ctypes.data,
                                    du.ctypes.data)
    if rc:
        raise ValueError(f"oracle_source_grad failed ({rc})")
    return dx, du[:, :p.D]


def target_grad(x, u, z, v, spec, ell, idx, T=None, sigma=1.0, kappa=3.0):
    """dF/dz_j and dF/dv_j for the targets j in idx only."""
    p = _Pair(x, u, z, v, spec)
    T = _pose(np.eye(4) if T is None else T)
    idx = np.ascontiguousarray(np.asarray(idx, np.int64))
    k = idx.shape[0]
    dz = np.zeros((k, 3)); dv = np.zeros((k, max(p.D, 1)))
    rc = _load().oracle_target_grad(C.byref(p.X), C.byref(p.Z), C.byref(p.S), ell, sigma, kappa,
                                    T.ctypes.data, idx.ctypes.data, k, dz.ctypes.data,
                                    dv.ctypes.data)
    if rc:
        raise ValueError(f"oracle_target_grad failed ({rc})")
    return dz, dv[:, :p.D]
