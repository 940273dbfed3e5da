"""Write the oracle's full-size registrations to ``full_size_registrations.json``.

Workloads, each registered by the FP64 oracle from the identity with the
annealing of Sec. IV (Problem 1, eq. (1)):
  * stereo-outdoor: 30,000 + 30,000 points, 5 SE colour/gradient + 19 LIN
    class-probability features, lengthscale 0.95 -> 0.1;
  * RGB-D-indoor: 40,000 + 40,000 points, 5 SE features, 0.1 -> 0.05;
  * batched0 .. batched7: the first 8 of the 64 mixed pairs of the batched
    workload (N, M ~ U[2000, 60000], 5 SE + 19 LIN), each with its shape's
    schedule;
  * stereo_adaptive, rgbd_adaptive: the stereo and RGB-D pairs registered
    with the lengthscale as an optimisation variable (Sec. VI; stereo from
    0.95 with a floor of 0.1, RGB-D from 0.1 with a floor of 0.02).
Stored per workload: a SHA-256 of the generated inputs (so a test can tell
that it regenerated the same clouds), the parameters, the converged pose,
the report, and the per-iteration trace columns the GPU tests compare
(lengthscale, F, |P|, step length).

Only ``paper_2012_03683_amd.synth`` (seeded input generators, no registration
arithmetic) and ``oracle`` are called.  About 15 minutes on 8 cores for the
two single pairs, 30 more for the batched subset and 13 for the two adaptive
runs.

Usage: python tests/golden/make_full_size.py [stereo|rgbd ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2012_03683_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "full_size_registrations.json")

_BATCH = {}


def _batched(k):
    """Pair k of the 64-pair batched workload (each pair has its own seeds,
    so the first 8 are the same whatever the batch size)."""
    if not _BATCH:
        _BATCH.update(enumerate(synth.batched_pairs(seed=1004, batch=8)))
    return _BATCH[k]


WORKLOADS = {
    "stereo": ("synth.stereo_pair(seed=1001)", lambda: synth.stereo_pair(seed=1001)),
    "rgbd": ("synth.rgbd_pair(seed=1002)", lambda: synth.rgbd_pair(seed=1002)),
}
for _k in range(8):
    WORKLOADS[f"batched{_k}"] = (f"synth.batched_pairs(seed=1004, batch=64)[{_k}]", lambda k=_k: _batched(k))
WORKLOADS["stereo_adaptive"] = WORKLOADS["stereo"]
WORKLOADS["rgbd_adaptive"] = WORKLOADS["rgbd"]

# parameters that replace the generator's defaults
OVERRIDES = {
    "stereo_adaptive": dict(ell_init=0.95, ell_min=0.1, max_iter=4000, ell_mode=1),
    "rgbd_adaptive": dict(ell_init=0.1, ell_min=0.02, max_iter=4000, ell_mode=1),
}


def input_hash(p) -> str:
    """SHA-256 over the four input arrays (float32, C order) and the spec."""
    h = hashlib.sha256()
    for a in (p.x, p.u, p.z, p.v):
        a = np.ascontiguousarray(a, dtype=np.float32)
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    h.update(json.dumps(p.spec, sort_keys=True).encode())
    return h.hexdigest()


def run(name):
    desc, make = WORKLOADS[name]
    p = make()
    params = dict(p.align, **OVERRIDES.get(name, {}))
    t0 = time.time()
    T, rep, tr = oracle.align(p.x, p.u, p.z, p.v, p.spec, params)
    sec = time.time() - t0
    print(f"{name}: {rep} in {sec:.0f} s", flush=True)
    return {
        "generator": desc,
        "input_sha256": input_hash(p),
        "points": [int(p.x.shape[0]), int(p.z.shape[0])],
        "spec": p.spec,
        "params": params,
        "T": T.tolist(),
        "report": rep,
        "trace": {
            "ell": tr[:, 1].tolist(),
            "F": tr[:, 2].tolist(),
            "n_pairs": [int(v) for v in tr[:, 6]],
            "tau": tr[:, 4].tolist(),
        },
        "oracle_seconds": round(sec, 1),
        "oracle_threads": oracle.num_threads(),
    }


def main(names):
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            out = json.load(fh)
    for name in names:
        out[name] = run(name)
        with open(OUT, "w") as fh:
            json.dump(out, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
