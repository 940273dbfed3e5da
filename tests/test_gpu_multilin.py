"""Several LIN feature blocks (eqs. (6)-(7): the feature kernel is the
product of the blocks' kernels).  The library folds the LIN blocks into
their tensor product, <u1 (x) u2, v1 (x) v2> = <u1, v1> <u2, v2>, and runs
them as one LIN block of prod(dims) columns; the backward takes the chain
rule back to each block.  Compared with the FP64 oracle, which multiplies
the blocks' inner products pair by pair: |P| exact, F and the gradient
within 1e-5, every backward output within 1e-5 of its scale."""
import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import assert_eval_matches, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPECS = {
    "se5_lin4_lin3": [synth.se_block(5, 0.2), synth.lin_block(4), synth.lin_block(3)],
    "lin2_se2_lin3_lin4": [synth.lin_block(2), synth.se_block(2, 0.3), synth.lin_block(3), synth.lin_block(4)],
}


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


def _cmp(g, o, name, rel=1e-5):
    g = g.double().cpu().numpy()
    scale = np.max(np.abs(o)) if o.size else 0.0
    err = np.abs(g - o)
    bound = rel * np.abs(o) + rel * 0.1 * scale + 1e-12
    assert not np.any(err > bound), f"{name}: {(err > bound).sum()} off, worst {np.max(err - bound):.3e}"


@pytest.mark.parametrize("name", list(SPECS))
def test_folded_lin_blocks_forward_and_backward(cvo, name):
    spec = SPECS[name]
    p = synth.random_pair(41, 2600, 2400, spec, extent=0.8)
    T = synth.random_motion(np.random.default_rng(7), 1.5, 0.02)
    X, Z, U, V = to_dev(p, torch)
    for ell in (0.08, 0.15):
        g = cvo.cvo_evaluate(X, Z, T, ell, U, V, spec)
        o = oracle.evaluate(p.x, p.u, p.z, p.v, spec, ell, T=T)
        print(name, ell, "|P|", g["n_pairs"], flush=True)
        assert_eval_matches(g, o, what=f"{name} ell={ell}")
        assert g["curv"] == pytest.approx(o["phi2"], rel=1e-4)
    b = cvo.cvo_inner_product_backward(X, Z, T, 0.1, 0.5, U, V, spec)
    ob = oracle.backward(p.x, p.u, p.z, p.v, spec, 0.1, T=T)
    _cmp(b["dX"], 0.5 * ob["dx"], "dX")
    _cmp(b["dZ"], 0.5 * ob["dz"], "dZ")
    _cmp(b["dU"], 0.5 * ob["du"], "dU")
    _cmp(b["dV"], 0.5 * ob["dv"], "dV")
    assert b["dell"] == pytest.approx(0.5 * ob["dell"], rel=1e-5)


def test_folded_lin_blocks_registration(cvo):
    """A registration with two LIN blocks converges where the oracle's does."""
    spec = SPECS["se5_lin4_lin3"]
    p = synth.random_pair(42, 1500, 1400, spec, extent=0.6, noise=0.01)
    X, Z, U, V = to_dev(p, torch)
    prm = dict(ell_init=0.2, ell_min=0.1, max_iter=800)
    Tg, rg, _ = cvo.cvo_align(X, Z, U, V, spec, prm)
    To, ro, _ = oracle.align(p.x, p.u, p.z, p.v, spec, prm)
    from gpu_util import pose_error
    ang, tr = pose_error(Tg, To)
    print("two LIN blocks: gpu", rg, "oracle", ro, "deviation", ang, tr, flush=True)
    assert rg["status"] == ro["status"] == oracle.CONVERGED
    assert ang < 1e-4 and tr < 1e-4


def test_tensor_product_too_wide_is_rejected(cvo):
    spec = [synth.lin_block(8), synth.lin_block(9)]        # 72 columns
    p = synth.random_pair(43, 100, 100, spec)
    X, Z, U, V = to_dev(p, torch)
    with pytest.raises(cvo.CvoError) as err:
        cvo.cvo_evaluate(X, Z, np.eye(4), 0.1, U, V, spec)
    assert err.value.code == cvo.CVO_ERR_UNSUPPORTED
