"""The project's autotuner of bin (grid cell) and tile (query cluster) sizes.

It times the pair pass over a search space of view shapes and keeps the
fastest, both as the one-shot shape and as the shape of the evaluation's
density class, which adaptive registrations (plain and batched) then use.
Whatever it picks changes speed, not results: evaluations match the FP64
oracle (exact |P|), and registrations with autotuned class shapes match
plain registrations and the oracle's converged poses (1e-4 rad / 1e-4 m).
Choices persist through a tuning file."""
import os

import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import assert_eval_matches, pose_error, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


@pytest.fixture
def clean(cvo):
    base = cvo.cvo_get_tuning()
    cvo.cvo_clear_tuning()
    yield
    cvo.cvo_clear_tuning()
    cvo.cvo_set_tuning(**base)


def test_autotune_choice_changes_speed_not_results(cvo, clean):
    p = synth.rgbd_pair(seed=1002, n=12000)
    X, Z, U, V = to_dev(p, torch)
    base = cvo.cvo_get_tuning()
    chosen = cvo.cvo_autotune(X, Z, p.T_gt, 0.1, U, V, p.spec)
    print("autotune chose", chosen, flush=True)
    assert chosen["cluster_max"] in (16, 32, 64) and chosen["cell_factor"] in (0.35, 0.5, 1.0)
    assert chosen["cluster_factor"] in (0.3, 0.5, 1.0, 1.5) and chosen["cluster_rule"] == 1
    assert chosen["adaptive"] == base["adaptive"] and chosen["unroll"] == base["unroll"]
    assert cvo.cvo_get_tuning() == chosen
    g = cvo.cvo_evaluate(X, Z, p.T_gt, 0.1, U, V, p.spec)
    o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, 0.1, T=p.T_gt)
    assert_eval_matches(g, o, what="autotuned")
    # a second call for the same size / layout / lengthscale class is cached
    cvo.cvo_set_tuning(**base)
    assert cvo.cvo_autotune(X, Z, p.T_gt, 0.1, U, V, p.spec) == chosen


def test_autotuned_class_shapes_drive_batched_registrations(cvo, clean, tmp_path):
    """Tune the stereo layout's density classes on the full stereo pair
    (ell 0.95: dense, 0.3: middle, 0.12: sparse), save and reload the table,
    then register reduced stereo pairs batched and plain: the registrations
    take their view shapes from the table, and agree with each other and
    with the oracle."""
    st = synth.stereo_pair(seed=1001)
    X, Z, U, V = to_dev(st, torch)
    for ell in (0.95, 0.3, 0.12):
        print("autotune stereo ell", ell, cvo.cvo_autotune(X, Z, st.T_gt, ell, U, V, st.spec), flush=True)
    path = os.path.join(str(tmp_path), "tuning.txt")
    cvo.cvo_save_tuning(path)
    text = open(path).read()
    print(text, flush=True)
    assert text.startswith("cvo-tuning 1") and text.count("\nclass ") >= 2
    cvo.cvo_clear_tuning()
    cvo.cvo_load_tuning(path)
    cvo.cvo_set_tuning(adaptive=1)
    pairs = [synth.stereo_pair(seed=1001 + 10 * k, n=2500 + 500 * k) for k in range(3)]
    prm = [dict(q.align, ell_min=0.2, max_iter=1500) for q in pairs]
    tens = [to_dev(q, torch) for q in pairs]
    cvo.cvo_set_profiling(False)
    Tb, rb = cvo.cvo_align_batched(tens, pairs[0].spec, prm)
    tim = cvo.cvo_get_timing()
    print("batched with tuned shapes", tim, flush=True)
    assert tim["tuned_view_shapes"] > 0
    for k, (q, t) in enumerate(zip(pairs, tens)):
        Tp, rp, _ = cvo.cvo_align(*t, q.spec, prm[k])
        ang, tr = pose_error(Tb[k], Tp)
        assert rb[k]["status"] == rp["status"] == cvo.CVO_CONVERGED
        assert ang < 1e-4 and tr < 1e-4
    To, ro, _ = oracle.align(pairs[0].x, pairs[0].u, pairs[0].z, pairs[0].v, pairs[0].spec, prm[0])
    ang, tr = pose_error(Tb[0], To)
    print("batched vs oracle", ang, tr, flush=True)
    assert ro["status"] == oracle.CONVERGED and ang < 1e-4 and tr < 1e-4


def test_tuning_file_rejects_garbage(cvo, clean, tmp_path):
    path = os.path.join(str(tmp_path), "bad.txt")
    with open(path, "w") as fh:
        fh.write("cvo-tuning 1\nclass 0 2 48 0.5 0.5 1\n")   # 48 points per cluster is not allowed
    with pytest.raises(cvo.CvoError):
        cvo.cvo_load_tuning(path)
    with open(path, "w") as fh:
        fh.write("not a tuning file\n")
    with pytest.raises(cvo.CvoError):
        cvo.cvo_load_tuning(path)
    with pytest.raises(cvo.CvoError):
        cvo.cvo_load_tuning(os.path.join(str(tmp_path), "missing.txt"))
