"""The batched form: many pairs of uneven sizes registered in one
device-resident, graph-replayed loop must give the per-pair results of
separate plain registrations (and of the oracle on a subset)."""
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


def _dev(q):
    d = torch.device("cuda:0")
    return (torch.from_numpy(q.x).to(d), torch.from_numpy(q.z).to(d), torch.from_numpy(q.u).to(d),
            torch.from_numpy(q.v).to(d))


def test_batched_matches_plain_and_oracle(cvo):
    pairs = synth.batched_pairs(seed=1004, batch=6, lo=1500, hi=4000)
    for q in pairs:
        q.align = dict(q.align, ell_min=max(q.align["ell_min"], 0.2) if "stereo" in q.name else q.align["ell_min"])
    tens = [_dev(q) for q in pairs]
    prm = [q.align for q in pairs]
    Tb, rb = cvo.cvo_align_batched(tens, pairs[0].spec, prm)
    for k, (q, t) in enumerate(zip(pairs, tens)):
        Tp, rp, _ = cvo.cvo_align(*t, q.spec, q.align)
        ang, tr = pose_error(Tb[k], Tp)
        print(q.name, rb[k]["iterations"], rp["iterations"], ang, tr)
        assert rb[k]["status"] == rp["status"] == cvo.CVO_CONVERGED
        assert ang < 1e-4 and tr < 1e-4
        if k < 2:
            To, ro, _ = oracle.align(q.x, q.u, q.z, q.v, q.spec, q.align)
            ang, tr = pose_error(Tb[k], To)
            assert ro["status"] == oracle.CONVERGED
            assert ang < 1e-4 and tr < 1e-4


def test_batched_with_empty_and_fixed_pairs(cvo):
    a = synth.tiny_cube(seed=5, n=1200)
    b = synth.tiny_cube(seed=6, n=900)
    ta, tb = _dev(a), _dev(b)
    empty = (ta[0][:0], tb[1], ta[2][:0], tb[3])
    prm = [dict(a.align), dict(b.align, max_iter=20), dict(a.align)]
    Ts, rs = cvo.cvo_align_batched([ta, tb, empty], a.spec, prm)
    assert rs[2]["status"] == cvo.CVO_NO_OVERLAP
    np.testing.assert_array_equal(Ts[2], np.eye(4))
    Ta, ra, _ = cvo.cvo_align(*ta, a.spec, a.align)
    Tb_, rb_, _ = cvo.cvo_align(*tb, b.spec, dict(b.align, max_iter=20))
    assert rs[0]["iterations"] == 50 and rs[1]["iterations"] == 20
    for T1, T2 in ((Ts[0], Ta), (Ts[1], Tb_)):
        ang, tr = pose_error(T1, T2)
        assert ang < 1e-9 and tr < 1e-9


def test_batched_full_size_pairs_match_plain(cvo):
    """The first 8 pairs of the 64-pair batched workload at their real sizes
    (N, M ~ U[2000, 60000], mixed stereo / RGB-D, 5 SE + 19 LIN): one batched
    call against 8 plain registrations (poses within 1e-4 rad / 1e-4 m), and
    one oracle evaluation at the final pose of the two smallest pairs (exact
    |P|, F and gradient within 1e-5 of their absolute sums)."""
    from gpu_util import assert_eval_matches
    pairs = synth.batched_pairs(seed=1004, batch=8)
    tens = [_dev(q) for q in pairs]
    prm = [q.align for q in pairs]
    print("sizes", [(q.x.shape[0], q.z.shape[0]) for q in pairs], flush=True)
    Tb, rb = cvo.cvo_align_batched(tens, pairs[0].spec, prm)
    for k, (q, t) in enumerate(zip(pairs, tens)):
        Tp, rp, _ = cvo.cvo_align(*t, q.spec, q.align)
        ang, tr = pose_error(Tb[k], Tp)
        print(q.name, rb[k]["iterations"], rp["iterations"], ang, tr, flush=True)
        assert rb[k]["status"] == rp["status"] == cvo.CVO_CONVERGED
        assert rb[k]["final_ell"] == rp["final_ell"]
        assert ang < 1e-4 and tr < 1e-4
    small = sorted(range(len(pairs)), key=lambda k: pairs[k].x.shape[0] * pairs[k].z.shape[0])[:2]
    for k in small:
        q = pairs[k]
        ell = rb[k]["final_ell"]
        g = cvo.cvo_evaluate(*tens[k][:2], Tb[k], ell, *tens[k][2:], q.spec)
        o = oracle.evaluate(q.x, q.u, q.z, q.v, q.spec, ell, T=Tb[k])
        assert_eval_matches(g, o, what=q.name)
