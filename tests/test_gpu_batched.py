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


@pytest.fixture(scope="module")
def batch64(cvo):
    """The full batched workload: 64 mixed stereo / RGB-D pairs, N and M ~
    U[2000, 60000], 5 SE + 19 LIN, registered in one batched call."""
    print("generating the 64 pairs", flush=True)
    pairs = synth.batched_pairs(seed=1004, batch=64)
    tens = [_dev(q) for q in pairs]
    print("batched registration of 64 pairs", flush=True)
    Tb, rb = cvo.cvo_align_batched(tens, pairs[0].spec, [q.align for q in pairs])
    return pairs, tens, Tb, rb


def test_batched_64_pairs_match_plain(cvo, batch64):
    """Every one of the 64 pairs: the batched result equals a plain
    registration's (same status and final lengthscale, poses within
    1e-4 rad / 1e-4 m)."""
    pairs, tens, Tb, rb = batch64
    worst = (0.0, 0.0)
    for k, (q, t) in enumerate(zip(pairs, tens)):
        Tp, rp, _ = cvo.cvo_align(*t, q.spec, q.align)
        ang, tr = pose_error(Tb[k], Tp)
        worst = (max(worst[0], ang), max(worst[1], tr))
        assert rb[k]["status"] == rp["status"] == cvo.CVO_CONVERGED, q.name
        assert rb[k]["final_ell"] == rp["final_ell"], q.name
        assert ang < 1e-4 and tr < 1e-4, (q.name, ang, tr)
    print("64 pairs: largest deviation from plain", worst, flush=True)


def test_batched_subset_matches_oracle_registrations(cvo, batch64):
    """Pairs 0-7 of the batched run against the oracle's converged
    registrations of the same pairs (golden/full_size_registrations.json,
    written by golden/make_full_size.py from the oracle alone): inputs hash
    to what the oracle ran on, same status and final lengthscale, poses
    within 1e-4 rad / 1e-4 m."""
    import importlib.util
    import json
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("make_full_size", os.path.join(here, "golden", "make_full_size.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(here, "golden", "full_size_registrations.json")) as fh:
        golden = json.load(fh)
    pairs, tens, Tb, rb = batch64
    for k in range(8):
        g = golden[f"batched{k}"]
        assert mod.input_hash(pairs[k]) == g["input_sha256"], k
        ang, tr = pose_error(Tb[k], np.array(g["T"]))
        print(pairs[k].name, "batched", rb[k]["iterations"], "oracle", g["report"]["iterations"],
              "pose deviation", ang, tr, flush=True)
        assert rb[k]["status"] == g["report"]["status"] == cvo.CVO_CONVERGED
        assert rb[k]["final_ell"] == g["report"]["final_ell"]
        assert ang < 1e-4 and tr < 1e-4
