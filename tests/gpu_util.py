"""Shared helpers for the GPU parity tests (tolerances, tensor upload)."""
import numpy as np

# Tolerance for F and each gradient component: |a - oracle| <= 1e-5 *
# max(|oracle|, A), A the oracle's sum of |per-pair term| (condition-aware
# relative error; near a stationary point the gradient itself tends to 0).
REL = 1e-5


def close(a, o, A, rel=REL):
    return abs(a - o) <= rel * max(abs(o), A)


def assert_eval_matches(g, o, rel=REL, what=""):
    assert g["n_pairs"] == o["n_pairs"], f"{what}: |P| {g['n_pairs']} != {o['n_pairs']}"
    assert close(g["F"], o["F"], o["absF"], rel), f"{what}: F {g['F']!r} vs {o['F']!r}"
    for k in range(6):
        assert close(g["grad"][k], o["grad"][k], o["absgrad"][k], rel), \
            f"{what}: grad[{k}] {g['grad'][k]!r} vs {o['grad'][k]!r} (A={o['absgrad'][k]!r})"


def to_dev(p, torch):
    dev = torch.device("cuda:0")
    X = torch.from_numpy(np.ascontiguousarray(p.x)).to(dev)
    Z = torch.from_numpy(np.ascontiguousarray(p.z)).to(dev)
    D = p.D
    U = torch.from_numpy(np.ascontiguousarray(p.u)).to(dev) if D else None
    V = torch.from_numpy(np.ascontiguousarray(p.v)).to(dev) if D else None
    return X, Z, U, V


def pose_error(Ta, Tb):
    E = np.linalg.inv(Tb) @ Ta
    ang = float(np.arccos(np.clip((np.trace(E[:3, :3]) - 1.0) / 2.0, -1.0, 1.0)))
    return ang, float(np.linalg.norm(E[:3, 3]))
