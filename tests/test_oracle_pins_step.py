"""Pins for the oracle parts that set the GPU tolerances and drive every
iterate: the absolute sums A_F, A_omega, A_v (eq. (7) term by term), one
ascent step (direction G^-1 g for the kinetic-energy metric, the Newton step
along it with the displacement clamp, the SE(3) exponential), the second
moments S_j, and clouds whose metric is degenerate.

Each check compares the oracle with something it does not contain: closed
forms derived by hand (tests/golden), a numpy brute force over the pairs of
tiny clouds, numpy's linear solve, scipy's matrix exponential, the
triangle inequality and rigid-motion covariance.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2012_03683_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
INF = float("inf")


def _hat(xi):
    w, v = xi[:3], xi[3:]
    W = np.zeros((4, 4))
    W[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    W[:3, 3] = v
    return W


def _golden_case(case):
    D = sum(b["dim"] for b in case["spec"])
    u = np.array(case["u"], np.float64).reshape(len(case["x"]), D)
    v = np.array(case["v"], np.float64).reshape(len(case["z"]), D)
    T = np.vstack([np.array(case["T"], np.float64), [0, 0, 0, 1]])
    return oracle.evaluate(case["x"], u, case["z"], v, case["spec"], case["ell"], T=T, kappa=case["kappa"])


# ------------------------------------------------------------ absolute sums
def test_abs_sums_of_single_pairs_equal_the_magnitudes():
    """One pair: every absolute sum is the magnitude of its value."""
    g = json.load(open(GOLD))
    for case in g["pairs"]:
        r = _golden_case(case)
        assert r["absF"] == abs(case["F"]) or r["absF"] == pytest.approx(abs(case["F"]), rel=1e-13)
        np.testing.assert_allclose(r["absgrad"], np.abs(case["grad"]), rtol=1e-13, atol=1e-300)
        np.testing.assert_array_equal(r["absgrad"], np.abs(r["grad"]))
        assert r["absF"] == abs(r["F"])


def test_abs_sums_closed_forms():
    """Hand-derived sums: two sources whose gradient terms cancel exactly (the
    sums do not), and a LIN block with a negative weight."""
    for case in json.load(open(GOLD))["abs_sums"]:
        r = _golden_case(case)
        assert r["n_pairs"] == case["n_pairs"], case["name"]
        assert r["F"] == pytest.approx(case["F"], rel=1e-13), case["name"]
        np.testing.assert_allclose(r["grad"], case["grad"], rtol=1e-13, atol=1e-15)
        assert r["absF"] == pytest.approx(case["absF"], rel=1e-13), case["name"]
        np.testing.assert_allclose(r["absgrad"], case["absgrad"], rtol=1e-13, atol=1e-15)
        assert r["dF_dell"] == pytest.approx(case["dF_dell"], rel=1e-13), case["name"]


def _brute_terms(p, ell, T, kappa, sigma=1.0):
    """Every in-cutoff pair's weight and difference vector, by numpy
    broadcasting over all N x M pairs (tiny clouds only)."""
    x = p.x.astype(np.float64)
    z = p.z.astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    d = x[:, None, :] - z[None, :, :]
    s = np.sum(d * d, axis=2)
    keep = s <= (kappa * ell) ** 2
    c = np.ones(s.shape)
    off = 0
    for b in p.spec:
        u = p.u[:, off:off + b["dim"]].astype(np.float64)
        v = p.v[:, off:off + b["dim"]].astype(np.float64)
        if b["kind"] == "se":
            e = u[:, None, :] - v[None, :, :]
            c *= b["sigma"] ** 2 * np.exp(-np.sum(e * e, axis=2) / (2 * b["ell"] ** 2))
        else:
            c *= u @ v.T
        off += b["dim"]
    w = np.where(keep, c * sigma ** 2 * np.exp(-s / (2 * ell * ell)), 0.0)
    zxd = np.cross(np.broadcast_to(z[None], d.shape), d)
    return w, d, zxd, keep


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_abs_sums_match_brute_force_and_bound_the_values(seed):
    """A_F = sum |w|, A_omega = ell^-2 sum |w||z' x d|, A_v = ell^-2 sum |w||d|
    against a numpy brute force, with LIN features of both signs; and the
    triangle inequality |value| <= A for F and every gradient component."""
    rng = np.random.default_rng(seed)
    spec = [synth.se_block(3, 0.5), synth.lin_block(4)]
    p = synth.random_pair(seed, 45, 40, spec, extent=0.3, noise=0.05)
    p.u[:, 3:] = rng.normal(size=(45, 4)).astype(np.float32)
    p.v[:, 3:] = rng.normal(size=(40, 4)).astype(np.float32)
    T = oracle.exp_se3(rng.normal(size=6) * 0.03)
    ell = 0.12
    r = oracle.evaluate(p.x, p.u, p.z, p.v, spec, ell, T=T)
    w, d, zxd, keep = _brute_terms(p, ell, T, 3.0)
    assert r["n_pairs"] == int(keep.sum()) > 50
    assert np.any(w < 0) and np.any(w > 0)
    aw = np.abs(w)[..., None]
    A_om = np.sum(aw * np.abs(zxd), axis=(0, 1)) / ell ** 2
    A_v = np.sum(aw * np.abs(d), axis=(0, 1)) / ell ** 2
    assert r["absF"] == pytest.approx(np.abs(w).sum(), rel=1e-12)
    np.testing.assert_allclose(r["absgrad"], np.r_[A_om, A_v], rtol=1e-12)
    assert abs(r["F"]) < r["absF"]
    assert np.all(np.abs(r["grad"]) <= r["absgrad"])


def test_abs_sum_of_F_is_F_when_every_weight_is_positive():
    """SE blocks only: every weight is positive, so A_F equals F (same terms,
    same order)."""
    p = synth.random_pair(4, 300, 280, [synth.se_block(5, 0.2)], extent=0.5)
    r = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, 0.1, T=np.eye(4))
    assert r["n_pairs"] > 300
    assert r["absF"] == r["F"]
    assert np.all(np.abs(r["grad"]) <= r["absgrad"])


# ------------------------------------------------------------ one ascent step
def _kinetic_metric_numpy(T, z):
    """G = (1/M) sum_j J_j^T J_j with J_j = [-[z'_j]_x, I], plus
    mu = 1e-6 (mean |z'|^2 + 1e-12) on the rotation block."""
    zt = z.astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    G = np.zeros((6, 6))
    for p in zt:
        J = np.zeros((3, 6))
        J[:, :3] = -np.array([[0, -p[2], p[1]], [p[2], 0, -p[0]], [-p[1], p[0], 0]])
        J[:, 3:] = np.eye(3)
        G += J.T @ J
    G /= zt.shape[0]
    G[:3, :3] += 1e-6 * (np.mean(np.sum(zt * zt, axis=1)) + 1e-12) * np.eye(3)
    return G


def _one_step(p, ell, T0, metric, lam=1.0, kappa=3.0):
    prm = dict(ell_init=ell, ell_min=ell, max_iter=1, fixed_iters=True, metric=metric, step_lambda=lam,
               kappa=kappa)
    T1, rep, tr = oracle.align(p.x, p.u, p.z, p.v, p.spec, prm, T_init=T0)
    ev = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T0, kappa=kappa)
    g = ev["grad"]
    d = np.linalg.solve(_kinetic_metric_numpy(T0, p.z), g) if metric == oracle.METRIC_KINETIC else g.copy()
    phi2 = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T0, kappa=kappa, direction=d)["phi2"]
    tau_n = (g @ d) / (-phi2) if phi2 < 0 else INF
    tau_c = lam * ell / (np.linalg.norm(d[:3]) * ev["r_max"] + np.linalg.norm(d[3:]))
    tau = min(tau_n, tau_c)
    return T1, rep, tr, dict(g=g, d=d, phi2=phi2, tau_n=tau_n, tau_c=tau_c, tau=tau, ev=ev)


CASES = {
    # near alignment at a moderate lengthscale: the Newton step is the shorter
    "newton": dict(misalign=(0.5, 0.01), ell=0.3, lam=1.0),
    # far from alignment at a small lengthscale: the displacement clamp binds
    "clamp": dict(misalign=(6.0, 0.25), ell=0.08, lam=1.0),
    # a small clamp factor: the clamp binds even near alignment
    "tight_clamp": dict(misalign=(0.5, 0.01), ell=0.3, lam=0.02),
}


@pytest.mark.parametrize("metric", [oracle.METRIC_KINETIC, oracle.METRIC_IDENTITY])
@pytest.mark.parametrize("case", list(CASES))
def test_first_ascent_step_follows_the_rule(case, metric):
    """One iteration of the ascent against the rule rebuilt outside the
    oracle: d = G^-1 g by numpy's solve (G built in numpy), tau_N = g.d / -phi''
    (phi'' along d from an oracle evaluation), tau_C = lam ell / (|d_w| r_max +
    |d_v|), tau = min, and T1 = expm(hat(tau d)) T0 by scipy."""
    c = CASES[case]
    p = synth.tiny_cube(seed=1000, n=600)
    rng = np.random.default_rng(7)
    T0 = p.T_gt @ synth.random_motion(rng, *c["misalign"])
    T1, rep, tr, ref = _one_step(p, c["ell"], T0, metric, lam=c["lam"])
    assert rep["iterations"] == 1 and tr.shape[0] == 1
    row = tr[0]
    assert row[1] == c["ell"]
    assert row[6] == ref["ev"]["n_pairs"]
    assert row[3] == pytest.approx(np.linalg.norm(ref["g"]), rel=1e-14)
    assert row[7] == pytest.approx(ref["phi2"], rel=1e-9, abs=1e-12 * abs(ref["phi2"]))
    assert row[4] == pytest.approx(ref["tau"], rel=1e-9)
    expect = scipy.linalg.expm(_hat(ref["tau"] * ref["d"])) @ T0
    np.testing.assert_allclose(T1, expect, rtol=0, atol=1e-12)
    binding = "newton" if ref["tau_n"] < ref["tau_c"] else "clamp"
    assert binding == ("newton" if case == "newton" else "clamp"), (ref["tau_n"], ref["tau_c"])


def test_step_is_not_newton_where_the_curvature_is_positive():
    """Far out on the kernel's tails F is convex along d (phi'' >= 0): tau_N is
    +inf and the clamp alone sets the step."""
    x = np.array([[0.0, 0.0, 0.0]], np.float32)
    z = np.array([[0.28, 0.0, 0.0]], np.float32)   # s = 0.0784 = 7.84 ell^2: beyond the inflexion at ell
    p = synth.Pair("tail", x, np.zeros((1, 0), np.float32), z, np.zeros((1, 0), np.float32), [], np.eye(4), 0.1)
    T1, rep, tr, ref = _one_step(p, 0.1, np.eye(4), oracle.METRIC_IDENTITY)
    assert ref["phi2"] > 0 and ref["tau_n"] == INF
    assert tr[0, 4] == pytest.approx(ref["tau_c"], rel=1e-12)
    # the clamp moves the point by exactly lambda ell (pure translation here)
    assert np.linalg.norm(T1[:3, 3]) == pytest.approx(0.1, rel=1e-12)


# ------------------------------------------------------------ second moments S_j
def _moments_brute(p, ell, T, idx):
    w, d, _, _ = _brute_terms(p, ell, T, 3.0)
    S = np.zeros((len(idx), 6))
    for q, j in enumerate(idx):
        for i in range(p.x.shape[0]):
            if w[i, j] == 0.0:
                continue
            o = np.outer(d[i, j], d[i, j]) * w[i, j]
            S[q] += [o[0, 0], o[0, 1], o[0, 2], o[1, 1], o[1, 2], o[2, 2]]
    return S


def test_second_moments_match_a_double_loop():
    """S_j = sum_i w_ij d_ij d_ij^T (xx, xy, xz, yy, yz, zz) for every target of
    a 20-point pair, off-diagonals included."""
    p = synth.random_pair(5, 20, 20, [synth.se_block(2, 0.4), synth.lin_block(3)], extent=0.15, noise=0.04)
    T = oracle.exp_se3([0.05, -0.03, 0.02, 0.01, -0.02, 0.015])
    idx = np.arange(20)
    W, Dm, S, cnt = oracle.target_moments(p.x, p.u, p.z, p.v, p.spec, 0.1, idx, T=T)
    Sb = _moments_brute(p, 0.1, T, idx)
    assert cnt.sum() > 60
    assert np.all(np.abs(Sb[:, [1, 2, 4]]).sum(0) > 0)
    np.testing.assert_allclose(S, Sb, rtol=1e-12, atol=1e-15 * np.abs(Sb).max())


def test_second_moments_rotate_as_a_tensor():
    """Moving both clouds by a signed permutation R_G (exact in float32) maps
    each S_j to R_G S_j R_G^T: fixes where each off-diagonal entry goes."""
    p = synth.random_pair(6, 30, 25, [synth.se_block(3, 0.5)], extent=0.2, noise=0.05)
    RG = np.array([[0.0, 0.0, -1.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    G = np.eye(4)
    G[:3, :3] = RG
    T = np.eye(4)
    T[:3, 3] = [0.0625, -0.03125, 0.015625]
    Tg = G @ T @ G.T
    idx = np.arange(25)
    _, _, S, c1 = oracle.target_moments(p.x, p.u, p.z, p.v, p.spec, 0.1, idx, T=T)
    xg = (p.x @ RG.T).astype(np.float32)
    zg = (p.z @ RG.T).astype(np.float32)
    _, _, Sg, c2 = oracle.target_moments(xg, p.u, zg, p.v, p.spec, 0.1, idx, T=Tg)
    np.testing.assert_array_equal(c1, c2)

    def full(s):
        return np.array([[s[0], s[1], s[2]], [s[1], s[3], s[4]], [s[2], s[4], s[5]]])

    for a, b in zip(S, Sg):
        np.testing.assert_allclose(full(b), RG @ full(a) @ RG.T, rtol=1e-12, atol=1e-14 * np.abs(a).max())


# ------------------------------------------------------------ degenerate moving clouds
def test_single_point_clouds_converge_to_the_translation():
    """One point in each cloud: the rotation is fixed only by the metric's
    regulariser, so the ascent moves z onto x by a translation (closed form
    T = (I, x - z))."""
    x = np.array([[0.3, -0.2, 1.5]], np.float32)
    z = np.array([[0.25, -0.17, 1.45]], np.float32)
    p = synth.Pair("one", x, np.zeros((1, 0), np.float32), z, np.zeros((1, 0), np.float32), [], np.eye(4), 0.1)
    prm = dict(ell_init=0.1, ell_min=0.1, max_iter=200, eps_rot=1e-10, eps_trans=1e-10)
    T, rep, tr = oracle.align(x, None, z, None, [], prm)
    assert rep["status"] == oracle.CONVERGED
    np.testing.assert_allclose(T[:3, :3] @ z[0].astype(np.float64) + T[:3, 3], x[0], atol=1e-7)
    np.testing.assert_allclose(T[:3, :3], np.eye(3), atol=1e-6)


def test_collinear_cloud_recovers_the_shift():
    """A moving cloud on a line (rotation about the line undetermined): the
    ascent still recovers a shift of the line's copy and leaves the free
    rotation at zero."""
    t = np.arange(7, dtype=np.float64) * 0.08
    z = np.stack([t, 0.5 + 0 * t, 2.0 + 0 * t], 1)
    shift = np.array([0.01, 0.02, -0.015])
    x = (z + shift).astype(np.float32)
    prm = dict(ell_init=0.1, ell_min=0.1, max_iter=500, eps_rot=1e-10, eps_trans=1e-10)
    T, rep, tr = oracle.align(x, None, z.astype(np.float32), None, [], prm)
    assert rep["status"] == oracle.CONVERGED
    np.testing.assert_allclose(T[:3, 3] + (T[:3, :3] - np.eye(3)) @ z.mean(0), shift, atol=1e-6)
    np.testing.assert_allclose(T[:3, :3], np.eye(3), atol=1e-5)
