"""The allocation-free entry point, cvo_evaluate_noalloc, against
cvo_evaluate: two calls in a row through the C ABI (a full-size stereo pair,
then a smaller RGB-D pair, so the second call reuses the fixed scratch the
first one left behind), each compared with cvo_evaluate on the same input to
the parity bar (|P| exact, F and gradient within 1e-5 of the larger of the
value and its absolute sum), plus the size limit."""
import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import assert_eval_matches, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


def _bar(got, ref, o, what):
    """got vs ref (the existing entry point), with the oracle's absolute sums
    as the scale of each component."""
    scale = dict(o)
    scale["n_pairs"] = ref["n_pairs"]
    scale["F"] = ref["F"]
    scale["grad"] = ref["grad"]
    assert_eval_matches(got, scale, what=what)
    assert got["curv"] == pytest.approx(ref["curv"], rel=1e-5, abs=1e-12)
    assert got["dF_dell"] == pytest.approx(ref["dF_dell"], rel=1e-5, abs=1e-12)


def test_noalloc_matches_evaluate_on_two_calls(cvo):
    big = synth.stereo_pair(seed=1001)
    small = synth.rgbd_pair(seed=1002, n=10000)
    cases = [(big, big.T_gt, 0.5), (small, np.eye(4), 0.1)]
    devs = [to_dev(p, torch) for p, _, _ in cases]
    print("noalloc: stereo 30000+30000 at ell 0.5, then rgbd 10000+10000 at ell 0.1", flush=True)
    got = [cvo.cvo_evaluate_noalloc(X, Z, T, ell, U, V, p.spec)
           for (p, T, ell), (X, Z, U, V) in zip(cases, devs)]
    ref = [cvo.cvo_evaluate(X, Z, T, ell, U, V, p.spec)
           for (p, T, ell), (X, Z, U, V) in zip(cases, devs)]
    for (p, T, ell), g, r in zip(cases, got, ref):
        o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T)
        same = all(np.array_equal(np.asarray(g[k]), np.asarray(r[k])) for k in g)
        print(p.name, "|P|", g["n_pairs"], "bitwise equal to cvo_evaluate:", same, flush=True)
        _bar(g, r, o, f"{p.name} noalloc vs evaluate")
        assert g["n_pairs"] == o["n_pairs"]


def test_noalloc_after_evaluate_and_empty_cloud(cvo):
    """The fixed scratch holds whatever the last call left: a call after the
    arena path, and one with an empty cloud, still match."""
    p = synth.tiny_cube(seed=1000)
    X, Z, U, V = to_dev(p, torch)
    r = cvo.cvo_evaluate(X, Z, np.eye(4), p.ell, U, V, p.spec)
    g = cvo.cvo_evaluate_noalloc(X, Z, np.eye(4), p.ell, U, V, p.spec)
    o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, p.ell)
    _bar(g, r, o, "tiny cube")
    e = cvo.cvo_evaluate_noalloc(X[:0], Z, np.eye(4), p.ell, U[:0], V, p.spec)
    assert e["n_pairs"] == 0 and e["F"] == 0.0


def test_noalloc_rejects_clouds_beyond_the_limit(cvo):
    """More points than the fixed scratch is sized for: rejected on the host
    before any device work, with the limit in the message."""
    n = 65537
    X = torch.zeros((n, 3), dtype=torch.float32, device="cuda:0")
    Z = torch.zeros((10, 3), dtype=torch.float32, device="cuda:0")
    with pytest.raises(cvo.CvoError) as err:
        cvo.cvo_evaluate_noalloc(X, Z, np.eye(4), 0.1)
    assert err.value.code == cvo.CVO_ERR_INVALID_ARGUMENT
    assert "65536" in str(err.value)
