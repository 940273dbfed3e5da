"""GPU parity of one pair pass (F, gradient, curvature, dF/dell, |P|) against
the FP64 oracle, through the C ABI.  |P| must match exactly; F and the
gradient within 1e-5 of max(|value|, sum of |terms|)."""
import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import REL, assert_eval_matches, close, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


def _run(cvo, p, T, ell, kappa=3.0, sigma=1.0):
    X, Z, U, V = to_dev(p, torch)
    g = cvo.cvo_evaluate(X, Z, T, ell, U, V, p.spec, sigma=sigma, kappa=kappa)
    o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T, sigma=sigma, kappa=kappa)
    return g, o


def test_tiny_cube_identity(cvo):
    p = synth.tiny_cube()
    g, o = _run(cvo, p, np.eye(4), 0.1)
    print("tiny_cube |P|", g["n_pairs"], "F", g["F"], o["F"])
    assert_eval_matches(g, o, what="tiny_cube")
    assert g["curv"] == pytest.approx(o["phi2"], rel=1e-4)
    assert g["dF_dell"] == pytest.approx(o["dF_dell"], rel=1e-4)
    assert g["r_max"] == pytest.approx(o["r_max"], rel=1e-12)
    assert g["i_theta"] == pytest.approx(o["i_theta"], rel=REL)


def test_tiny_cube_at_truth(cvo):
    p = synth.tiny_cube()
    g, o = _run(cvo, p, p.T_gt, 0.1)
    assert_eval_matches(g, o, what="tiny_cube@T_gt")


SPECS = {
    "geometric": [],
    "se5": [synth.se_block(5, 0.2)],
    "se5_lin19": [synth.se_block(5, 0.2), synth.lin_block(19)],
    "lin32": [synth.lin_block(32)],
    "se2_se3": [synth.se_block(2, 0.3), synth.se_block(3, 0.5, sigma=1.3)],
    "lin3": [synth.lin_block(3)],
    "se7_lin1": [synth.se_block(7, 0.4), synth.lin_block(1)],
    # the wide compiled kernels: 16 and 32 SE columns, 64 LIN columns
    "se12": [synth.se_block(12, 0.6)],
    "se20_lin19": [synth.se_block(20, 0.8), synth.lin_block(19)],
    "se16_lin32": [synth.se_block(16, 0.7), synth.lin_block(32)],
    "lin40": [synth.lin_block(40)],
}


@pytest.mark.parametrize("name", list(SPECS))
@pytest.mark.parametrize("nm", [(3001, 2777), (1, 1), (64, 65), (700, 129)])
def test_ragged_layouts(cvo, name, nm):
    n, m = nm
    spec = SPECS[name]
    p = synth.random_pair(7 + n + m, n, m, spec, extent=1.0 if n > 100 else 0.05, noise=0.05)
    T = synth.random_motion(np.random.default_rng(n), 2.0, 0.03)
    g, o = _run(cvo, p, T, 0.08)
    assert_eval_matches(g, o, what=f"{name} {nm}")
    if o["n_pairs"]:
        assert g["curv"] == pytest.approx(o["phi2"], rel=1e-3, abs=1e-4 * abs(o["phi2"]) + 1e-9)


@pytest.mark.parametrize("kappa", [1.0, 2.0, 5.0, float("inf")])
def test_cutoff_values(cvo, kappa):
    p = synth.random_pair(11, 900, 800, [synth.se_block(5, 0.2)], extent=0.6)
    T = synth.random_motion(np.random.default_rng(2), 1.0, 0.02)
    g, o = _run(cvo, p, T, 0.07, kappa=kappa)
    assert_eval_matches(g, o, what=f"kappa={kappa}")


def test_sigma(cvo):
    p = synth.random_pair(12, 500, 400, [synth.se_block(5, 0.2)], extent=0.5)
    g, o = _run(cvo, p, np.eye(4), 0.08, sigma=2.5)
    assert_eval_matches(g, o, what="sigma")


def test_exact_ties_and_near_boundary_pairs(cvo):
    """Pairs at s = rc^2 exactly and at rc^2 (1 +/- 2^-k): the GPU count must
    equal the FP64 definition's."""
    rng = np.random.default_rng(19)
    ell, kappa = 0.125, 2.0
    rc = kappa * ell
    x = rng.uniform(-0.3, 0.3, (300, 3)).astype(np.float32)
    dirs = rng.normal(size=(300, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    zs = []
    for k in range(8, 53):
        for sgn in (-1, 1):
            i = rng.integers(0, 300)
            zs.append(x[i].astype(np.float64) + dirs[k % 300] * rc * np.sqrt(1 + sgn * 2.0 ** -k))
    for i in range(20):
        e = np.zeros(3)
        e[i % 3] = rc * (1 if i % 2 else -1)
        zs.append(x[i].astype(np.float64) + e)
    z = np.array(zs).astype(np.float32)
    p = synth.Pair("ties", x, np.zeros((300, 0), np.float32), z, np.zeros((len(z), 0), np.float32), [],
                   np.eye(4), ell)
    for T in (np.eye(4), synth.random_motion(np.random.default_rng(5), 0.5, 0.01)):
        g, o = _run(cvo, p, T, ell, kappa=kappa)
        assert_eval_matches(g, o, what="ties")


def test_far_from_origin(cvo):
    """Clouds 2 km from the origin: relative coordinates keep the FP32 kernel accurate."""
    p = synth.random_pair(13, 1500, 1400, [synth.se_block(5, 0.2)], extent=1.0)
    off = np.array([2000.0, -1500.0, 800.0], np.float32)
    p.x = p.x + off
    p.z = p.z + off
    T = np.eye(4)
    g, o = _run(cvo, p, T, 0.08)
    assert_eval_matches(g, o, what="far")


def test_duplicates_and_single_cell(cvo):
    """Many coincident points (one octree block holding far more than a
    cluster) and a cloud inside one grid cell."""
    rng = np.random.default_rng(3)
    base = rng.uniform(-0.01, 0.01, (5, 3))
    x = np.repeat(base, 200, axis=0).astype(np.float32)
    z = (x + rng.normal(0, 1e-3, x.shape)).astype(np.float32)
    u = rng.uniform(0, 1, (x.shape[0], 5)).astype(np.float32)
    v = rng.uniform(0, 1, (z.shape[0], 5)).astype(np.float32)
    p = synth.Pair("dups", x, u, z, v, [synth.se_block(5, 0.3)], np.eye(4), 0.05)
    g, o = _run(cvo, p, np.eye(4), 0.05)
    assert_eval_matches(g, o, what="dups")


def test_no_overlap_and_empty(cvo):
    p = synth.random_pair(14, 100, 100, [], extent=0.1)
    p.z = p.z + np.float32(100.0)
    g, o = _run(cvo, p, np.eye(4), 0.1)
    assert g["n_pairs"] == o["n_pairs"] == 0 and g["F"] == 0.0
    X = torch.zeros((0, 3), device="cuda")
    Z = torch.from_numpy(p.z).cuda()
    F, n = cvo.cvo_inner_product(X, Z, np.eye(4), 0.1)
    assert F == 0.0 and n == 0
    assert cvo.cvo_metric(X, Z, np.eye(4), 0.1) == 0.0


def test_inner_product_gradient_metric_agree(cvo):
    p = synth.tiny_cube(n=1500)
    X, Z, U, V = to_dev(p, torch)
    e = cvo.cvo_evaluate(X, Z, p.T_gt, 0.1, U, V, p.spec)
    F, n = cvo.cvo_inner_product(X, Z, p.T_gt, 0.1, U, V, p.spec)
    F2, g, n2 = cvo.cvo_gradient(X, Z, p.T_gt, 0.1, U, V, p.spec)
    m = cvo.cvo_metric(X, Z, p.T_gt, 0.1, U, V, p.spec)
    assert F == e["F"] == F2 and n == n2 == e["n_pairs"]
    np.testing.assert_array_equal(g, e["grad"])
    assert m == pytest.approx(F / np.sqrt(1500 * 1500), rel=1e-15)


def test_bitwise_reproducible(cvo):
    p = synth.random_pair(15, 4000, 3500, [synth.se_block(5, 0.2), synth.lin_block(19)], extent=1.0)
    X, Z, U, V = to_dev(p, torch)
    a = cvo.cvo_evaluate(X, Z, np.eye(4), 0.1, U, V, p.spec)
    b = cvo.cvo_evaluate(X, Z, np.eye(4), 0.1, U, V, p.spec)
    assert a["F"] == b["F"] and np.array_equal(a["grad"], b["grad"]) and a["curv"] == b["curv"]


def test_remark_unit_indicator(cvo):
    """Remark before eq. (10): well-separated identical clouds give i_theta = 1."""
    ax = np.arange(6, dtype=np.float32)
    x = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    u = np.random.default_rng(0).uniform(0, 1, (x.shape[0], 5)).astype(np.float32)
    p = synth.Pair("grid", x, u, x.copy(), u.copy(), [synth.se_block(5, 0.2)], np.eye(4), 0.1)
    X, Z, U, V = to_dev(p, torch)
    assert cvo.cvo_metric(X, Z, np.eye(4), 0.1, U, V, p.spec) == 1.0


def test_invalid_arguments_raise(cvo):
    p = synth.tiny_cube(n=100)
    X, Z, U, V = to_dev(p, torch)
    with pytest.raises(cvo.CvoError):
        cvo.cvo_evaluate(X, Z, np.eye(4), -1.0, U, V, p.spec)
    bad = np.eye(4)
    bad[0, 0] = 2.0
    with pytest.raises(cvo.CvoError):
        cvo.cvo_evaluate(X, Z, bad, 0.1, U, V, p.spec)
    Xn = X.clone()
    Xn[3, 1] = float("nan")
    with pytest.raises(cvo.CvoError):
        cvo.cvo_evaluate(Xn, Z, np.eye(4), 0.1, U, V, p.spec)
    with pytest.raises(ValueError):
        cvo.cvo_evaluate(X, Z, np.eye(4), 0.1, None, None, p.spec)


def test_point_count_limit_rejected(cvo):
    """Point counts outside [0, 2^30) are rejected on the host, before any
    device work (the buffers here are small real ones; nothing reads them)."""
    import ctypes as C
    p = synth.tiny_cube(n=100)
    X, Z, U, V = to_dev(p, torch)
    cx, cz, keep, sp = cvo._prep(X, Z, U, V, p.spec)
    kp = cvo.cvo_kernel_params(0.1, 1.0, 3.0)
    Tp = cvo._pose(np.eye(4))
    lib, h = cvo.load_library(), cvo.handle()
    for bad in (1 << 30, (1 << 31) + 5, -1):
        for which in ("X", "Z"):
            cx.n, cz.n = X.shape[0], Z.shape[0]
            (cx if which == "X" else cz).n = bad
            F, n = C.c_double(), C.c_int64()
            st = lib.cvo_inner_product(h, C.byref(cx), C.byref(cz), C.byref(sp), C.byref(kp), Tp.ctypes.data,
                                       C.byref(F), C.byref(n))
            assert st == cvo.CVO_ERR_INVALID_ARGUMENT, (bad, which, st)
            assert "point count out of range" in lib.cvo_last_error(h).decode(), (bad, which)
    del keep
    # the handle still works afterwards
    assert cvo.cvo_inner_product(X, Z, np.eye(4), 0.1, U, V, p.spec)[1] > 0


@pytest.mark.parametrize("dims", [(50, 60, 50), (160, 160, 160)], ids=["150k", "4096k"])
def test_large_cloud_self_pairs_closed_form(cvo, dims):
    """Clouds of 150,000 and 4,096,000 points (more than the reduction covers
    with one query per thread, so its blocks loop over queries; the larger one
    also coarsens the grid to the library's cell cap): a unit lattice and a
    copy of it moved by < 0.07 per point, at ell = 0.1, cutoff 0.3.  Every
    point pairs with its own copy only, so |P| = N and F, the gradient and
    dF/dell are plain sums over the N offsets (eq. (7) with no features),
    evaluated here in FP64."""
    rng = np.random.default_rng(77)
    g = np.stack(np.meshgrid(*(np.arange(k) for k in dims), indexing="ij"), -1).reshape(-1, 3)
    x = g.astype(np.float32)
    z = (g + rng.uniform(-0.04, 0.04, g.shape)).astype(np.float32)
    assert x.shape[0] == dims[0] * dims[1] * dims[2]
    ell = 0.1
    X, Z = torch.from_numpy(x).cuda(), torch.from_numpy(z).cuda()
    r = cvo.cvo_evaluate(X, Z, np.eye(4), ell, None, None, [])
    d = x.astype(np.float64) - z.astype(np.float64)
    s = (d * d).sum(1)
    w = np.exp(-s / (2 * ell * ell))
    zz = z.astype(np.float64)
    v_terms = w[:, None] * d / ell ** 2
    om_terms = w[:, None] * np.cross(zz, d) / ell ** 2
    assert r["n_pairs"] == x.shape[0]
    assert r["F"] == pytest.approx(w.sum(), rel=1e-6)
    grad = np.asarray(r["grad"])
    ref = np.concatenate([om_terms.sum(0), v_terms.sum(0)])
    scale = np.concatenate([np.abs(om_terms).sum(0), np.abs(v_terms).sum(0)])
    assert np.all(np.abs(grad - ref) <= 1e-5 * scale), (grad, ref)
    assert r["dF_dell"] == pytest.approx((w * s).sum() / ell ** 3, rel=1e-5)
