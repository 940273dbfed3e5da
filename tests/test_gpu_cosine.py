"""GPU parity of the exact cosine of the angle between f_X and the moved f_Z
(eq. (9)) against the FP64 oracle, through the C ABI: the three inner
products within 1e-5 of max(|value|, sum of |terms|), the cosine within the
error those bounds allow, and the misalignment sweep of Sec. III-C."""
import numpy as np
import pytest

import oracle
from paper_2012_03683_amd import synth

from gpu_util import REL, close, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvo():
    import paper_2012_03683_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    m.load_library()
    return m


def _check(cvo, p, T, ell, kappa=3.0):
    X, Z, U, V = to_dev(p, torch)
    g = cvo.cvo_cosine(X, Z, T, ell, U, V, p.spec, kappa=kappa)
    o = oracle.cosine(p.x, p.u, p.z, p.v, p.spec, ell, T=T, kappa=kappa)
    # abs sums of each inner product bound the rounding of its GPU value
    A = [oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell, T=T, kappa=kappa)["absF"],
         oracle.evaluate(p.x, p.u, p.x, p.u, p.spec, ell, kappa=kappa)["absF"],
         oracle.evaluate(p.z, p.v, p.z, p.v, p.spec, ell, kappa=kappa)["absF"]]
    for k, name in enumerate(("F_XZ", "F_XX", "F_ZZ")):
        assert close(g[k + 1], o[k + 1], A[k]), f"{p.name} {name}: {g[k + 1]!r} vs {o[k + 1]!r}"
    # first-order propagation of those bounds into F_XZ / sqrt(F_XX F_ZZ)
    tol = REL * (A[0] / np.sqrt(o[2] * o[3]) + abs(o[0]) * 0.5 * (A[1] / o[2] + A[2] / o[3]))
    assert abs(g[0] - o[0]) <= tol, f"{p.name} cos {g[0]!r} vs {o[0]!r} (tol {tol:.3g})"
    return g, o


def test_cosine_tiny_cube(cvo):
    p = synth.tiny_cube()
    for T in (np.eye(4), p.T_gt):
        g, o = _check(cvo, p, T, 0.1)
        print("tiny cube cos", g[0], o[0])


def test_cosine_stereo_and_learned_features(cvo):
    p = synth.stereo_pair(seed=1001, n=3000)
    _check(cvo, p, p.T_gt, 0.5)
    _check(cvo, p, np.eye(4), 0.95)
    q = synth.learned_batch(seed=1003, batch=1, n=2000)[0]
    _check(cvo, q, q.T_eval, q.ell)


@pytest.mark.parametrize("which,ell", [("stereo", 0.5), ("rgbd", 0.1)])
def test_cosine_full_size(cvo, which, ell):
    """The full stereo (30k + 30k, 5 SE + 19 LIN) and RGB-D (40k + 40k, 5 SE)
    pairs at their true poses: the three inner products and the cosine."""
    p = synth.stereo_pair(seed=1001) if which == "stereo" else synth.rgbd_pair(seed=1002)
    g, o = _check(cvo, p, p.T_gt, ell)
    print(which, "cos", g[0], o[0], flush=True)


def test_cosine_sweep_peaks_at_alignment(cvo):
    """Fig. 3 of Sec. III-C: a stereo-shaped cloud rotated and translated
    against itself; cos(theta) and i_theta match the oracle at every sample and
    are largest (cos = 1) at zero error."""
    p0 = synth.stereo_pair(seed=1001, n=3000)
    p = synth.Pair("self", p0.x, p0.u, p0.x.copy(), p0.u.copy(), p0.spec, np.eye(4), 0.3)
    X, Z, U, V = to_dev(p, torch)
    axis = np.array([0.1, 0.98, 0.15]) / np.linalg.norm([0.1, 0.98, 0.15])
    cos_g, ind_g = [], []
    for th in np.deg2rad([0.0, 0.5, 1.0, 2.0, 5.0]):
        T = oracle.exp_se3(np.r_[th * axis, 0, 0, 0])
        g, o = _check(cvo, p, T, 0.3)
        cos_g.append(g[0])
        ind_g.append(cvo.cvo_metric(X, Z, T, 0.3, U, V, p.spec))
    assert cos_g[0] == 1.0
    assert np.all(np.diff(cos_g) < 0) and np.all(np.diff(ind_g) < 0)


def test_cosine_empty_cloud_is_zero(cvo):
    p = synth.tiny_cube(n=100)
    X, Z, U, V = to_dev(p, torch)
    c, fxz, fxx, fzz = cvo.cvo_cosine(X, Z[:0], np.eye(4), 0.1, U, V[:0], p.spec)
    assert c == 0.0 and fxz == 0.0 and fzz == 0.0 and fxx > 0.0
