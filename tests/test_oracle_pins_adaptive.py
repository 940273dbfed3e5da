"""Pins for the oracle's adaptive lengthscale (Sec. VI: the lengthscale as an
optimisation variable).

The reading: ell maximises the log-likelihood of the moved cloud under the
kernel mixture centred on X,
    J(T, ell) = sum_{j : W_j > 0} log W_j - 3 |Z+| log ell,
with W_j = sum_i w_ij over the pair set frozen at (T, ell); its stationary
point for fixed per-target residuals is ell^2 = sum_j r_j / (3 |Z+|).

Each check compares the oracle with something it does not contain: a
closed form (one source, Gaussian targets), numpy evaluations of J from its
definition, central differences of that numpy J, scipy's scalar maximiser,
the adaptive update rule rebuilt from oracle evaluations, and recovery of a
known transform.
"""
import numpy as np
import pytest
import scipy.optimize
from scipy.spatial.transform import Rotation

import oracle
from paper_2012_03683_amd import synth

INF = float("inf")


def _numpy_J(x, u, z, v, spec, ell, T, kappa, frozen_ell=None):
    """J from its definition by numpy broadcasting over all pairs.  The pair
    set is taken at frozen_ell (default: ell), the weights at ell."""
    x = np.asarray(x, np.float32).astype(np.float64)
    z = np.asarray(z, np.float32).astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    d = x[:, None, :] - z[None, :, :]
    s = np.sum(d * d, axis=2)
    fe = ell if frozen_ell is None else frozen_ell
    keep = s <= (kappa * fe) ** 2
    c = np.ones(s.shape)
    off = 0
    for b in spec:
        uu = np.asarray(u, np.float32)[:, off:off + b["dim"]].astype(np.float64)
        vv = np.asarray(v, np.float32)[:, off:off + b["dim"]].astype(np.float64)
        if b["kind"] == "se":
            e = uu[:, None, :] - vv[None, :, :]
            c *= b["sigma"] ** 2 * np.exp(-np.sum(e * e, axis=2) / (2 * b["ell"] ** 2))
        else:
            c *= uu @ vv.T
        off += b["dim"]
    W = np.sum(np.where(keep, c * np.exp(-s / (2 * ell * ell)), 0.0), axis=0)
    pos = W > 0
    return np.sum(np.log(W[pos])) - 3 * pos.sum() * np.log(ell), int(pos.sum())


def test_one_source_closed_form():
    """One source at the origin, targets ~ N(0, 0.2^2 I), no cutoff and no
    features: each target has one pair, so r_j = |z_j|^2 exactly,
    ell_ml^2 = mean |z|^2 / 3 whatever ell is, J = -sum |z|^2 / (2 ell^2) -
    3 M log ell and dJ/dell = sum |z|^2 / ell^3 - 3 M / ell."""
    rng = np.random.default_rng(3)
    z = rng.normal(0.0, 0.2, (400, 3)).astype(np.float32)
    x = np.zeros((1, 3), np.float32)
    r2 = np.sum(z.astype(np.float64) ** 2, axis=1)
    for ell in (0.05, 0.2, 0.7):
        o = oracle.ell_objective(x, None, z, None, [], ell, kappa=INF)
        assert o["n_plus"] == 400
        assert o["ell_ml"] == pytest.approx(np.sqrt(r2.mean() / 3), rel=1e-12)
        assert o["J"] == pytest.approx(-r2.sum() / (2 * ell * ell) - 1200 * np.log(ell), rel=1e-12)
        assert o["dJ_dell"] == pytest.approx(r2.sum() / ell ** 3 - 1200 / ell, rel=1e-12)
    # the sample estimate is near the generating scale
    assert abs(np.sqrt(r2.mean() / 3) - 0.2) < 0.02


@pytest.mark.parametrize("seed", [1, 2])
def test_J_matches_numpy_definition(seed):
    """Random clouds with an SE and a non-negative LIN block, cutoff kappa = 3,
    a general pose: J and |Z+| against the numpy definition."""
    spec = [synth.se_block(3, 0.5), synth.lin_block(4)]
    p = synth.random_pair(seed, 60, 55, spec, extent=0.3, noise=0.05)
    p.u[:, 3:] = np.abs(p.u[:, 3:])
    p.v[:, 3:] = np.abs(p.v[:, 3:])
    T = oracle.exp_se3(np.random.default_rng(seed).normal(size=6) * 0.03)
    for ell in (0.05, 0.1, 0.2):
        o = oracle.ell_objective(p.x, p.u, p.z, p.v, spec, ell, T=T)
        J, npos = _numpy_J(p.x, p.u, p.z, p.v, spec, ell, T, 3.0)
        assert o["n_plus"] == npos > 10
        assert o["J"] == pytest.approx(J, rel=1e-12, abs=1e-12 * abs(J))


def test_dJ_matches_frozen_set_central_difference():
    """dJ/dell against a central difference of the numpy J with the pair set
    frozen at ell (Richardson-extrapolated)."""
    spec = [synth.se_block(5, 0.4)]
    p = synth.random_pair(9, 80, 70, spec, extent=0.3, noise=0.04)
    T = synth.random_motion(np.random.default_rng(2), 1.0, 0.01)
    ell = 0.1

    def fd(h):
        jp, _ = _numpy_J(p.x, p.u, p.z, p.v, spec, ell + h, T, 3.0, frozen_ell=ell)
        jm, _ = _numpy_J(p.x, p.u, p.z, p.v, spec, ell - h, T, 3.0, frozen_ell=ell)
        return (jp - jm) / (2 * h)

    h = 1e-4
    rich = (4 * fd(h / 2) - fd(h)) / 3
    o = oracle.ell_objective(p.x, p.u, p.z, p.v, spec, ell, T=T)
    assert o["dJ_dell"] == pytest.approx(rich, rel=1e-7, abs=1e-7 * abs(o["J"]))


def test_fixed_point_is_the_maximiser():
    """No cutoff: iterating ell <- ell_ml converges to the maximiser of J over
    ell, found independently by scipy on the numpy J."""
    rng = np.random.default_rng(5)
    x = rng.normal(0.0, 0.3, (40, 3)).astype(np.float32)
    z = (x[rng.integers(0, 40, 150)] + rng.normal(0.0, 0.05, (150, 3))).astype(np.float32)
    T = np.eye(4)
    res = scipy.optimize.minimize_scalar(lambda e: -_numpy_J(x, None, z, None, [], e, T, INF)[0],
                                         bounds=(0.005, 1.0), method="bounded",
                                         options={"xatol": 1e-12})
    ell = 0.5
    for _ in range(500):
        nxt = oracle.ell_objective(x, None, z, None, [], ell, kappa=INF)["ell_ml"]
        if abs(nxt - ell) < 1e-14:
            break
        ell = nxt
    assert ell == pytest.approx(res.x, rel=1e-6)
    assert abs(oracle.ell_objective(x, None, z, None, [], ell, kappa=INF)["dJ_dell"]) < 1e-6 * 150 / ell
    # near the noise scale of the targets about their sources
    assert 0.03 < ell < 0.08


def test_targets_with_negative_weight_sums_are_left_out():
    """A LIN block of mixed sign: only targets with W_j > 0 count."""
    spec = [synth.lin_block(3)]
    p = synth.random_pair(4, 50, 45, spec, extent=0.25, noise=0.05)
    rng = np.random.default_rng(8)
    p.u[:] = rng.normal(size=p.u.shape).astype(np.float32)
    p.v[:] = rng.normal(size=p.v.shape).astype(np.float32)
    o = oracle.ell_objective(p.x, p.u, p.z, p.v, spec, 0.1)
    J, npos = _numpy_J(p.x, p.u, p.z, p.v, spec, 0.1, np.eye(4), 3.0)
    assert 0 < o["n_plus"] == npos < 45
    assert o["J"] == pytest.approx(J, rel=1e-12)


def _adaptive(ell0, ell_min, max_iter, **kw):
    return dict(ell_init=ell0, ell_min=ell_min, max_iter=max_iter, ell_mode=oracle.ELL_ADAPTIVE, **kw)


def test_adaptive_update_rule():
    """Each iteration sets ell to the maximum-likelihood lengthscale of the
    iteration's (T, ell) before the step, clamped to [ell_min, ell_init] and
    to a factor `decay` of ell.  Rebuilt for three iterations from oracle
    evaluations and one-iteration runs."""
    p = synth.tiny_cube(seed=1000, n=800)
    prm0 = _adaptive(0.3, 0.05, 1)
    T, ell = np.eye(4), 0.3
    for k in range(3):
        # runs are deterministic: the run of k + 1 iterations repeats the run
        # of k, so its last transition starts from (T, ell) of the latter
        Tk, rep, tr = oracle.align(p.x, p.u, p.z, p.v, p.spec, dict(prm0, max_iter=k + 1))
        assert tr[k, 1] == ell
        ml = oracle.ell_objective(p.x, p.u, p.z, p.v, p.spec, ell, T=T)["ell_ml"]
        lo, hi = max(0.98 * ell, 0.05), min(ell / 0.98, 0.3)
        expect = min(max(ml, lo), hi)
        assert rep["final_ell"] == pytest.approx(expect, rel=1e-15)
        T, ell = Tk, rep["final_ell"]


def test_adaptive_noise_free_recovery():
    """Z = T_gt^-1 X exactly: the adaptive run recovers T_gt, and its
    lengthscale falls to the floor (the residuals vanish at alignment)."""
    rng = np.random.default_rng(31)
    x = rng.uniform(-1.0, 1.0, (500, 3))
    u = rng.uniform(0, 1, (500, 5))
    T_gt = synth.random_motion(rng, 4.0, 0.08)
    Ti = np.linalg.inv(T_gt)
    z = x @ Ti[:3, :3].T + Ti[:3, 3]
    prm = _adaptive(0.3, 0.1, 2000, eps_rot=1e-9, eps_trans=1e-9)
    T, rep, tr = oracle.align(x, u, z, u, [synth.se_block(5, 0.3)], prm)
    assert rep["status"] == oracle.CONVERGED
    E = np.linalg.inv(T_gt) @ T
    assert np.linalg.norm(Rotation.from_matrix(E[:3, :3]).as_rotvec()) < 1e-5
    assert np.linalg.norm(E[:3, 3]) < 1e-5
    assert rep["final_ell"] == 0.1
    # every step moves ell by at most the clamp factor
    r = tr[1:, 1] / tr[:-1, 1]
    assert np.all(r >= 0.98 - 1e-15) and np.all(r <= 1 / 0.98 + 1e-15)


def test_adaptive_tiny_cube_recovers_motion():
    """The tiny cube with noise (Z = T_gt^-1 X + N(0, 0.01 m) per coordinate)
    from the identity, ell from 0.3 with a floor of 0.002: the adaptive run
    converges near T_gt, and ell settles above the floor at the noise scale
    (the targets' residuals about their sources), not at the floor."""
    p = synth.tiny_cube()
    T, rep, tr = oracle.align(p.x, p.u, p.z, p.v, p.spec, _adaptive(0.3, 0.002, 3000))
    assert rep["status"] == oracle.CONVERGED
    E = np.linalg.inv(p.T_gt) @ T
    assert np.rad2deg(np.linalg.norm(Rotation.from_matrix(E[:3, :3]).as_rotvec())) < 0.05
    assert np.linalg.norm(E[:3, 3]) < 2e-3
    assert 0.005 < rep["final_ell"] < 0.02
