"""GPU parity of the hand-written backward (dF/dX, dF/dZ, dF/dU, dF/dV,
dF/dell on the frozen pair set) against the FP64 oracle, identities that
hold at any size, finite differences through the autograd Function, and the
32-dim learned-feature workload (8 stereo-shaped pairs of 10k points)."""
import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


def _cmp(g, o, name, rel=1e-5):
    g = g.double().cpu().numpy() if hasattr(g, "cpu") else np.asarray(g)
    scale = np.max(np.abs(o)) if o.size else 0.0
    err = np.abs(g - o)
    bound = rel * np.abs(o) + rel * 0.1 * scale + 1e-12
    bad = err > bound
    assert not np.any(bad), f"{name}: {bad.sum()} elements off, worst {np.max(err - bound):.3e} (scale {scale:.3e})"


SPECS = {
    "geometric": [],
    "se5": [synth.se_block(5, 0.2)],
    "se5_lin19": [synth.se_block(5, 0.2), synth.lin_block(19)],
    "lin32": [synth.lin_block(32)],
    "se20_lin19": [synth.se_block(20, 0.8), synth.lin_block(19)],
    "lin40": [synth.lin_block(40)],
}


@pytest.mark.parametrize("name", list(SPECS))
def test_backward_matches_oracle(cvo, name):
    spec = SPECS[name]
    p = synth.random_pair(21, 2100, 1900, spec, extent=0.8)
    T = synth.random_motion(np.random.default_rng(4), 1.5, 0.02)
    X, Z, U, V = to_dev(p, torch)
    ell = 0.09
    gF = 0.75
    b = cvo.cvo_inner_product_backward(X, Z, T, ell, gF, U, V, spec)
    o = oracle.backward(p.x, p.u, p.z, p.v, spec, ell, T=T)
    _cmp(b["dX"], gF * o["dx"], "dX")
    _cmp(b["dZ"], gF * o["dz"], "dZ")
    if spec:
        _cmp(b["dU"], gF * o["du"], "dU")
        _cmp(b["dV"], gF * o["dv"], "dV")
    assert b["dell"] == pytest.approx(gF * o["dell"], rel=1e-5)


def test_backward_identities_on_gpu_outputs(cvo):
    """sum_i dF/dx_i = -v, sum_j R dF/dz_j = v, sum_i x_i x dF/dx_i = -omega."""
    p = synth.random_pair(22, 3000, 2800, [synth.se_block(5, 0.2), synth.lin_block(19)], extent=1.0)
    T = synth.random_motion(np.random.default_rng(5), 1.0, 0.02)
    X, Z, U, V = to_dev(p, torch)
    b = cvo.cvo_inner_product_backward(X, Z, T, 0.1, 1.0, U, V, p.spec)
    e = cvo.cvo_evaluate(X, Z, T, 0.1, U, V, p.spec)
    o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, 0.1, T=T)
    dx = b["dX"].double().cpu().numpy()
    dz = b["dZ"].double().cpu().numpy()
    A = np.max(o["absgrad"])
    np.testing.assert_allclose(dx.sum(0), -e["grad"][3:], atol=2e-5 * A)
    np.testing.assert_allclose((dz @ T[:3, :3].T).sum(0), e["grad"][3:], atol=2e-5 * A)
    np.testing.assert_allclose(np.cross(p.x.astype(np.float64), dx).sum(0), -e["grad"][:3], atol=2e-5 * A * 3)
    du = b["dU"].double().cpu().numpy()
    assert np.sum(p.u[:, 5:].astype(np.float64) * du[:, 5:]) == pytest.approx(e["F"], rel=2e-5)


def test_learned_feature_workload(cvo):
    """8 stereo-shaped pairs of 10k points with 32-dim L2-normalised LIN
    features at T = T_gt Exp(0.5 deg, 2 cm), ell = 0.3: forward F and the
    backward against the oracle -- every output in full for the first two
    pairs; for the other six, 64 sampled rows of each of dX, dU, dZ, dV and
    dF/dell against the oracle's pass."""
    pairs = synth.learned_batch(seed=1003, batch=8)
    rng = np.random.default_rng(0)
    for k, p in enumerate(pairs):
        X, Z, U, V = to_dev(p, torch)
        F, n = cvo.cvo_inner_product(X, Z, p.T_eval, p.ell, U, V, p.spec)
        b = cvo.cvo_inner_product_backward(X, Z, p.T_eval, p.ell, 1.0, U, V, p.spec)
        if k < 2:
            o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, p.ell, T=p.T_eval)
            assert n == o["n_pairs"]
            assert abs(F - o["F"]) <= 1e-5 * o["absF"]
            ob = oracle.backward(p.x, p.u, p.z, p.v, p.spec, p.ell, T=p.T_eval)
            _cmp(b["dX"], ob["dx"], "dX")
            _cmp(b["dZ"], ob["dz"], "dZ")
            _cmp(b["dU"], ob["du"], "dU")
            _cmp(b["dV"], ob["dv"], "dV")
            assert b["dell"] == pytest.approx(ob["dell"], rel=1e-5, abs=1e-5 * o["absF"] / p.ell)
        else:
            o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, p.ell, T=p.T_eval)
            assert n == o["n_pairs"]
            assert abs(F - o["F"]) <= 1e-5 * o["absF"]
            idx = rng.choice(p.x.shape[0], 64, replace=False)
            dx, du = oracle.source_grad(p.x, p.u, p.z, p.v, p.spec, p.ell, idx, T=p.T_eval)
            _cmp(b["dX"][idx], dx, f"dX sample {k}")
            _cmp(b["dU"][idx], du, f"dU sample {k}")
            jdx = rng.choice(p.z.shape[0], 64, replace=False)
            dz, dv = oracle.target_grad(p.x, p.u, p.z, p.v, p.spec, p.ell, jdx, T=p.T_eval)
            _cmp(b["dZ"][jdx], dz, f"dZ sample {k}")
            _cmp(b["dV"][jdx], dv, f"dV sample {k}")
            # dF/dell = sum w s / ell^3 on the frozen set (the oracle's pass)
            assert b["dell"] == pytest.approx(o["dF_dell"], rel=1e-5, abs=1e-5 * o["absF"] / p.ell)


@pytest.mark.parametrize("ell", [0.5, 0.1])
def test_full_size_stereo_backward_sampled(cvo, ell):
    """The stereo-outdoor pair at full size (30k + 30k points, 5 SE + 19 LIN)
    at its true pose, in a dense (ell = 0.5) and a sparse (ell = 0.1) band:
    64 sampled rows of each of dX, dU, dZ and dV against the oracle's per-row
    gradients, and dF/dell, F and |P| against the oracle's full evaluation."""
    p = synth.stereo_pair(seed=1001)
    X, Z, U, V = to_dev(p, torch)
    b = cvo.cvo_inner_product_backward(X, Z, p.T_gt, ell, 1.0, U, V, p.spec)
    F, n = cvo.cvo_inner_product(X, Z, p.T_gt, ell, U, V, p.spec)
    o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=p.T_gt)
    print("stereo backward ell", ell, "pairs", n, flush=True)
    assert n == o["n_pairs"] > 0
    assert abs(F - o["F"]) <= 1e-5 * o["absF"]
    assert b["dell"] == pytest.approx(o["dF_dell"], rel=1e-5, abs=1e-5 * o["absF"] / ell)
    rng = np.random.default_rng(5)
    idx = rng.choice(p.x.shape[0], 64, replace=False)
    dx, du = oracle.source_grad(p.x, p.u, p.z, p.v, p.spec, ell, idx, T=p.T_gt)
    _cmp(b["dX"][idx], dx, "dX sample")
    _cmp(b["dU"][idx], du, "dU sample")
    jdx = rng.choice(p.z.shape[0], 64, replace=False)
    dz, dv = oracle.target_grad(p.x, p.u, p.z, p.v, p.spec, ell, jdx, T=p.T_gt)
    _cmp(b["dZ"][jdx], dz, "dZ sample")
    _cmp(b["dV"][jdx], dv, "dV sample")


def test_autograd_function(cvo):
    p = synth.random_pair(23, 600, 500, [synth.se_block(5, 0.25)], extent=0.4)
    T = synth.random_motion(np.random.default_rng(6), 1.0, 0.01)
    X, Z, U, V = to_dev(p, torch)
    X.requires_grad_(True); Z.requires_grad_(True); U.requires_grad_(True); V.requires_grad_(True)
    ell = torch.tensor(0.12, dtype=torch.float64, requires_grad=True)
    F = cvo.CvoInnerProduct.apply(X, Z, U, V, T, ell, p.spec, 1.0, float("inf"))
    F.backward()
    o = oracle.backward(p.x, p.u, p.z, p.v, p.spec, 0.12, T=T, kappa=float("inf"))
    _cmp(X.grad, o["dx"], "autograd dX")
    _cmp(Z.grad, o["dz"], "autograd dZ")
    _cmp(U.grad, o["du"], "autograd dU")
    _cmp(V.grad, o["dv"], "autograd dV")
    assert ell.grad.item() == pytest.approx(o["dell"], rel=1e-5)
    # finite differences of the GPU forward on a few coordinates (no cutoff)
    h = 1e-3
    for i, c in ((3, 0), (17, 2), (101, 1)):
        Xp = X.detach().clone(); Xp[i, c] += h
        Xm = X.detach().clone(); Xm[i, c] -= h
        Fp = cvo.cvo_inner_product(Xp, Z.detach(), T, 0.12, U.detach(), V.detach(), p.spec, kappa=float("inf"))[0]
        Fm = cvo.cvo_inner_product(Xm, Z.detach(), T, 0.12, U.detach(), V.detach(), p.spec, kappa=float("inf"))[0]
        fd = (Fp - Fm) / (float(Xp[i, c]) - float(Xm[i, c]))
        assert X.grad[i, c].item() == pytest.approx(fd, rel=2e-3, abs=1e-3 * abs(fd) + 1e-4)


def _local_terms(xq, uq, pts, feats, ell, rc2, frozen, moving_is_source, T):
    """Sum of the LIN-kernel terms of one point against the other cloud over
    its pair set frozen at the base position (float64)."""
    if moving_is_source:
        d = xq[None, :] - pts                       # pts: transformed targets
    else:
        zt = xq @ T[:3, :3].T + T[:3, 3]
        d = pts - zt[None, :]                       # pts: sources
    s = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    return float(np.sum(np.where(frozen, (feats @ uq) * np.exp(-s / (2 * ell * ell)), 0.0)))


def test_learned_feature_finite_differences(cvo):
    """Central differences (h = 1e-3) on the learned-feature workload (all 8
    pairs of 10k + 10k points, 32 LIN, ell = 0.3, cutoff 3 ell): for 24
    random coordinates of each cloud's positions and features, the terms
    involving the moved point are re-summed in float64 over the pair set
    frozen at the base pose (the cutoff held fixed), and dF/dell from the
    oracle's F at ell +- h with the cutoff radius fixed; the GPU backward
    must agree within 1e-4 of the scale of its entries (the truncation
    error of the difference is ~(h / ell)^2 / 6 ~ 2e-6)."""
    pairs = synth.learned_batch(seed=1003, batch=8)
    rng = np.random.default_rng(1)
    h = 1e-3
    for k, p in enumerate(pairs):
        X, Z, U, V = to_dev(p, torch)
        b = cvo.cvo_inner_product_backward(X, Z, p.T_eval, p.ell, 1.0, U, V, p.spec)
        T, ell = p.T_eval, p.ell
        rc = 3.0 * ell
        rc2 = rc * rc
        x = p.x.astype(np.float64); z = p.z.astype(np.float64)
        u = p.u.astype(np.float64); v = p.v.astype(np.float64)
        zt = oracle.transform(T, p.z)
        gx = b["dX"].double().cpu().numpy(); gz = b["dZ"].double().cpu().numpy()
        gu = b["dU"].double().cpu().numpy(); gv = b["dV"].double().cpu().numpy()
        worst = 0.0
        for side in ("source", "target"):
            n = x.shape[0] if side == "source" else z.shape[0]
            for i in rng.choice(n, 24, replace=False):
                if side == "source":
                    base, feat, pts, feats, gpos, gfeat = x[i], u[i], zt, v, gx[i], gu[i]
                    d0 = base[None, :] - pts
                else:
                    base, feat, pts, feats, gpos, gfeat = z[i], v[i], x, u, gz[i], gv[i]
                    d0 = pts - oracle.transform(T, p.z[i:i + 1])
                s0 = (d0[:, 0] * d0[:, 0] + d0[:, 1] * d0[:, 1]) + d0[:, 2] * d0[:, 2]
                frozen = s0 <= rc2
                if not frozen.any():
                    continue
                src = side == "source"
                c = rng.integers(0, 3)
                e = np.zeros(3); e[c] = h
                fd = (_local_terms(base + e, feat, pts, feats, ell, rc2, frozen, src, T) -
                      _local_terms(base - e, feat, pts, feats, ell, rc2, frozen, src, T)) / (2 * h)
                scale = np.max(np.abs(gx if src else gz)) + 1e-30
                worst = max(worst, abs(gpos[c] - fd) / scale)
                assert abs(gpos[c] - fd) <= 1e-4 * scale, (k, side, i, c, gpos[c], fd)
                f = rng.integers(0, feat.shape[0])
                ef = np.zeros(feat.shape[0]); ef[f] = h
                fdf = (_local_terms(base, feat + ef, pts, feats, ell, rc2, frozen, src, T) -
                       _local_terms(base, feat - ef, pts, feats, ell, rc2, frozen, src, T)) / (2 * h)
                fscale = np.max(np.abs(gu if src else gv)) + 1e-30
                assert abs(gfeat[f] - fdf) <= 1e-4 * fscale, (k, side, i, f, gfeat[f], fdf)
        # lengthscale: the oracle's F at ell +- h with the cutoff radius fixed
        op = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell + h, T=T, kappa=rc / (ell + h))
        om = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell - h, T=T, kappa=rc / (ell - h))
        o0 = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T)
        if op["n_pairs"] == om["n_pairs"] == o0["n_pairs"]:
            fd = (op["F"] - om["F"]) / (2 * h)
            assert b["dell"] == pytest.approx(fd, rel=1e-4, abs=1e-4 * o0["absF"] / ell), (k, b["dell"], fd)
        print(f"pair {k}: worst position FD deviation {worst:.2e} of the gradient scale", flush=True)
