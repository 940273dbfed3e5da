"""Oracle parity of every view shape a registration switches to, at full size.

Registrations re-choose the query-cluster size and rule, the grid cell edge
and the cluster edge cap (as multiples of the cutoff radius) from the pair
density of their latest iteration; the dense-band shapes carry most of the
stereo workload's pairs.  Each shape is set by hand (adaptive off) and one-shot
evaluations of the full stereo-outdoor pair (30k + 30k, 5 SE + 19 LIN) at
ell = 0.95, 0.5, 0.25 and of the full RGB-D-indoor pair (40k + 40k, 5 SE) at
ell = 0.1 are compared with the FP64 oracle (eq. (7) and its gradient) at the
identity and at the true pose: |P| exact, F and the gradient within 1e-5,
the curvature and dF/dell within 1e-4 (both sum the FP32 second
moments)."""
import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import assert_eval_matches, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (points per cluster, cell edge / r_c, cluster edge cap / r_c, cluster
# rule): every chunk-cluster shape of the autotuner's search space (which
# holds the built-in density table's shapes), two octree shapes (the one-shot
# default and a dense one), and the finest cells allowed: a neighbourhood then
# spans more than 64 rows of cells, so the pass measures its rows in several
# batches
SHAPES = ([(cm, cell, cf, 1) for cm in (16, 32, 64) for cell in (0.35, 0.5, 1.0) for cf in (0.3, 0.5, 1.0, 1.5)]
          + [(16, 1.0, 0.5, 0), (64, 0.5, 0.5, 0), (32, 0.25, 1.0, 1)])


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


@pytest.fixture(scope="module")
def cases():
    """(pair, device tensors, [(T, ell, oracle evaluation)]), oracle computed once."""
    out = []
    st = synth.stereo_pair(seed=1001)
    rg = synth.rgbd_pair(seed=1002)
    for p, ells in ((st, (0.95, 0.5, 0.25)), (rg, (0.1,))):
        evals = []
        for ell in ells:
            for T in (np.eye(4), p.T_gt):
                print(f"oracle {p.name} ell={ell}", flush=True)
                evals.append((T, ell, oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T)))
        out.append((p, to_dev(p, torch), evals))
    return out


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{'chunk' if s[3] else 'octree'}{s[0]}_cell{s[1]}_clus{s[2]}"
                                               for s in SHAPES])
def test_view_shape_matches_oracle_at_full_size(cvo, cases, shape):
    base = cvo.cvo_get_tuning()
    try:
        cvo.cvo_set_tuning(adaptive=0, cluster_max=shape[0], cell_factor=shape[1], cluster_factor=shape[2],
                           cluster_rule=shape[3])
        for p, (X, Z, U, V), evals in cases:
            for T, ell, o in evals:
                what = f"{p.name} shape={shape} ell={ell} {'truth' if T is p.T_gt else 'identity'}"
                print(what, flush=True)
                g = cvo.cvo_evaluate(X, Z, T, ell, U, V, p.spec)
                assert_eval_matches(g, o, what=what)
                assert g["curv"] == pytest.approx(o["phi2"], rel=1e-4), what
                assert g["dF_dell"] == pytest.approx(o["dF_dell"], rel=1e-4), what
    finally:
        cvo.cvo_set_tuning(**base)
