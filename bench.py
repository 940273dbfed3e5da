"""Benchmark of the CVO hot path on one MI355X.

One step = one full registration of the stereo-outdoor pair (30,000 + 30,000
points, 5 SE colour/gradient + 19 LIN class-probability features,
lengthscale annealed 0.95 -> 0.1 until convergence) followed by the
alignment metric at the result: transform, grid/cluster preparation, pair
passes, reductions, ascent steps, annealing and the metric, all on the GPU.

Printed JSON line:
  value      kernel-pair evaluations per second over the whole job
             (sum of |P| over every evaluation / wall time of the steps)
  roofline   the pair-pass kernel against the VALU issue rate
             (256 CU x 64 lanes x 2.4 GHz = 39.3e12 lane-ops/s): algorithmic
             lane-ops per pair x pairs / summed HIP-event time of its launches
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample
  extra      registrations/s, the batched form vs a loop of plain calls, the
             backward form
Inputs are resident in device memory before the timed region starts.

roofline.traffic is the pair-pass kernel's HBM bytes per launch from
rocprofv3 FETCH_SIZE / WRITE_SIZE counters (profiles/pair_pass_traffic.json,
scaled by the same counters read on a plain copy: `--copy-calibration`); it is
null when the kernel source has changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_SLOTS = 256 * 64 * 2.4e9          # VALU lane-ops per second (non-packed issue)


def ops_per_pair(n_se, n_lin):
    """Algorithmic VALU lane-ops per in-cutoff pair of the forward pass, as the
    kernel's inner loop issues them: squared distance 6 (3 sub, 1 mul, 2 fma),
    cutoff test 1, exp2 4 (quarter rate), W and D 7 (1 add, 3 mul, 3 add; the
    FP64 conversion happens once per queue flush, not per pair), second
    moments S 6 (fma), pair count 1  = 25;  + 2 per SE column (sub, fma);
    + per LIN block: 1 fma per column, 1 add joining the dot's two FMA
    chains, 1 multiply of the weight.  5 SE + 19 LIN: 25 + 10 + 21 = 56.
    Loop control and the exact-recheck compare are not counted."""
    return 25 + 2 * n_se + (n_lin + 2 if n_lin else 0)


KERNEL_SOURCES = ("paper_2012_03683_amd/csrc/cvo_pairs.hip", "paper_2012_03683_amd/csrc/cvo_internal.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_pass_traffic.json")


def _code_only(text):
    """The source without comments, trailing blanks and empty lines, so that
    editing a comment does not invalidate counters taken on the same code."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per pair-pass launch from the committed counter summary, or
    None when it is missing or was taken on another version of the kernel."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def copy_calibration(nbytes=256 << 20, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters (run under rocprofv3 --pmc)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").uniform_()
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--batched", type=int, default=64,
                    help="pairs in the batched-vs-plain comparison of the extras (64 = the full batched workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration) and exit")
    ap.add_argument("--iteration-trace", default=None,
                    help="write the last timed registration's per-iteration trace (it, ell, F, |grad|, tau, "
                         "i_theta, |P|, curvature) to this text file, to match per-dispatch counters to "
                         "lengthscale bands")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; more than one is not supported (use --gpus 1)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    import paper_2012_03683_amd as cvo
    from paper_2012_03683_amd import synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    cvo.load_library()
    dev = torch.device("cuda:0")

    p = synth.stereo_pair(seed=1001)
    X = torch.from_numpy(p.x).to(dev)
    Z = torch.from_numpy(p.z).to(dev)
    U = torch.from_numpy(p.u).to(dev)
    V = torch.from_numpy(p.v).to(dev)
    params = dict(p.align)
    torch.cuda.synchronize()

    last_trace = []

    def step():
        T, rep, tr = cvo.cvo_align(X, Z, U, V, p.spec, params, trace=args.iteration_trace is not None)
        m = cvo.cvo_metric(X, Z, T, rep["final_ell"], U, V, p.spec)
        last_trace[:] = [tr]
        return T, rep, m

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    cvo.cvo_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        T, rep, m = step()
        reps.append((T, rep, m))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tim = cvo.cvo_get_timing()
    cvo.cvo_set_profiling(False)
    if args.iteration_trace is not None and last_trace and last_trace[0] is not None:
        np.savetxt(args.iteration_trace, last_trace[0])

    total_pairs = sum(r[1]["total_pairs"] for r in reps)
    # the metric call adds one more pass per step
    metric_pairs = 0
    for T, rep, m in reps:
        metric_pairs += cvo.cvo_inner_product(X, Z, T, rep["final_ell"], U, V, p.spec)[1]
    pairs = total_pairs + metric_pairs
    value = pairs / wall
    ms_step = 1e3 * wall / args.steps
    opp = ops_per_pair(5, 19)
    kernel_s = tim["pair_ms"] / 1e3
    # the library's pair count already holds every timed launch's |P|, the
    # metric passes included
    achieved = tim["pair_count"] * opp / kernel_s if kernel_s > 0 else 0.0
    evaluations = sum(r[1]["iterations"] + 1 for r in reps)   # ascent iterations + the metric pass
    T_last, rep_last, m_last = reps[-1]
    Eerr = np.linalg.inv(p.T_gt) @ T_last
    rot_err = float(np.degrees(np.arccos(np.clip((np.trace(Eerr[:3, :3]) - 1) / 2, -1, 1))))
    out = {
        "metric": "kernel-pair evals/s + registrations/s (F+se(3) grad) vs plain path, 1 MI355X",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic; W, D summed in f32 over <= 80 pairs per lane, then f64; "
                 "S in f32; f64 reduction, step and pose",
        "data": "synthetic (seeded stereo-outdoor generator; KITTI stand-in)",
        "config": {
            "workload": "stereo-outdoor pair, 30000+30000 points, 5 SE + 19 LIN features, "
                        "registration ell 0.95->0.1 to convergence + alignment metric",
            "points": [int(p.x.shape[0]), int(p.z.shape[0])],
            "feature_dim": int(p.D),
            "iterations_per_registration": int(rep_last["iterations"]),
            "pairs_per_registration": int(rep_last["total_pairs"]),
            "registrations_per_s": args.steps / wall,
            "status": int(rep_last["status"]),
            "final_ell": rep_last["final_ell"],
            "rot_err_deg_vs_truth": rot_err,
            "trans_err_m_vs_truth": float(np.linalg.norm(Eerr[:3, 3])),
            "i_theta": m_last,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_SLOTS / 1e12,
            "unit": "T lane-ops/s",
            "frac": achieved / PEAK_SLOTS,
            "traffic": measured_traffic(),
            "kernel": "pair_pass_kernel<5,19,0>",
            "ops_per_pair": opp,
            "kernel_pair_evals_per_s": tim["pair_count"] / kernel_s if kernel_s > 0 else 0.0,
            "avg_launch_ms": tim["pair_ms"] / max(tim["pair_launches"], 1),
            "launches": tim["pair_launches"],
            "evaluations": evaluations,
            "ms_per_evaluation": tim["pair_ms"] / max(evaluations, 1),
        },
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, rep_last)
    if not args.no_extra:
        out["extra"] = extras(cvo, torch, synth, dev, args.batched)
    print(json.dumps(out))


def cpu_baseline(p, rep):
    """The FP64 oracle on this host: one evaluation (F, gradient, curvature;
    brute force over all N x M candidate pairs) at every third lengthscale of
    the anneal, 0.95 * 0.98^(3 i) down to 0.1, on the same stereo pair."""
    import oracle
    ells = []
    ell = 0.95
    while ell >= 0.1:
        ells.append(ell)
        ell *= 0.98 ** 3
    pairs = 0
    t0 = time.perf_counter()
    for ell in ells:
        o = oracle.evaluate(p.x, p.u, p.z, p.v, p.spec, ell)
        pairs += o["n_pairs"]
    sec = time.perf_counter() - t0
    per_eval = sec / len(ells)
    return {
        "value": pairs / sec,
        "unit": "pair-evals/s",
        "cores": oracle.num_threads(),
        "candidates_per_s": len(ells) * p.x.shape[0] * p.z.shape[0] / sec,
        "kind": "oracle",
        "sample": f"{len(ells)} FP64 oracle evaluations (F, gradient, curvature; brute force over all "
                  f"{p.x.shape[0] * p.z.shape[0]:.1e} candidate pairs each) of the same stereo pair at the anneal's "
                  f"lengthscales 0.95*0.98^(3i), i = 0..{len(ells) - 1}: {sec:.1f} s",
        "registrations_per_s_est": 1.0 / (per_eval * max(1, rep["iterations"])),
    }


def extras(cvo, torch, synth, dev, nbatch):
    """Figures for the other workloads (each timed after one untimed run)."""
    ex = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    # RGB-D indoor: 40k + 40k points, 5 SE, ell 0.1 -> 0.05, then the metric
    q = synth.rgbd_pair(seed=1002)
    X, Z, U, V = (torch.from_numpy(a).to(dev) for a in (q.x, q.z, q.u, q.v))
    sec, (T, rep, _) = timed(lambda: cvo.cvo_align(X, Z, U, V, q.spec, q.align), 3)
    ex["rgbd_registration_ms"] = 1e3 * sec
    ex["rgbd_pair_evals_per_s"] = rep["total_pairs"] / sec
    ex["rgbd_iterations"] = int(rep["iterations"])
    # exact cosine of eq. (9) on the RGB-D pair at its registered pose (three pair passes)
    sec, cs = timed(lambda: cvo.cvo_cosine(X, Z, T, rep["final_ell"], U, V, q.spec), 5)
    ex["rgbd_cosine_ms"] = 1e3 * sec
    ex["rgbd_cosine_at_result"] = cs[0]
    # tiny cube: 2k + 2k points, 50 fixed ascent iterations at ell = 0.1
    q = synth.tiny_cube(seed=1000)
    X, Z, U, V = (torch.from_numpy(a).to(dev) for a in (q.x, q.z, q.u, q.v))
    sec, _ = timed(lambda: cvo.cvo_align(X, Z, U, V, q.spec, q.align), 5)
    ex["tiny_cube_50_iterations_ms"] = 1e3 * sec
    # adaptive lengthscale (the lengthscale as an optimisation variable):
    # stereo from 0.95 with a floor of 0.1, RGB-D from 0.1 with a floor of 0.02
    for name, q, prm in (("stereo", synth.stereo_pair(seed=1001), dict(ell_init=0.95, ell_min=0.1)),
                         ("rgbd", synth.rgbd_pair(seed=1002), dict(ell_init=0.1, ell_min=0.02))):
        X, Z, U, V = (torch.from_numpy(a).to(dev) for a in (q.x, q.z, q.u, q.v))
        prm = dict(prm, max_iter=4000, ell_mode=cvo.CVO_ELL_ADAPTIVE)
        sec, (T, rep, _) = timed(lambda: cvo.cvo_align(X, Z, U, V, q.spec, prm), 3)
        E = np.linalg.inv(q.T_gt) @ T
        ex[f"adaptive_{name}_registration_ms"] = 1e3 * sec
        ex[f"adaptive_{name}_iterations"] = int(rep["iterations"])
        ex[f"adaptive_{name}_final_ell"] = rep["final_ell"]
        ex[f"adaptive_{name}_rot_err_deg"] = float(np.degrees(np.arccos(np.clip((np.trace(E[:3, :3]) - 1) / 2, -1, 1))))
        ex[f"adaptive_{name}_trans_err_m"] = float(np.linalg.norm(E[:3, 3]))
    # batched form vs looping the plain path, on the batched workload (64
    # mixed pairs, N, M ~ U[2000, 60000]); first with the built-in density
    # table, then with view shapes autotuned per density class
    pairs = synth.batched_pairs(seed=1004, batch=nbatch)
    tens = [tuple(torch.from_numpy(a).to(dev) for a in (b.x, b.z, b.u, b.v)) for b in pairs]
    prm = [b.align for b in pairs]
    spec = pairs[0].spec

    def batched():
        return cvo.cvo_align_batched(tens, spec, prm)

    def plain():
        return [cvo.cvo_align(X, Z, U, V, spec, pr) for (X, Z, U, V), pr in zip(tens, prm)]

    def counted(fn):
        fn()
        torch.cuda.synchronize()
        cvo.cvo_set_profiling(False)   # resets the counters
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        c = cvo.cvo_get_timing()
        return sec, {k: c[k] for k in ("evaluations", "graph_launches", "graph_captures", "view_builds",
                                       "host_waits", "tuned_view_shapes")}

    cvo.cvo_clear_tuning()
    tb, cb = counted(batched)
    tp, cp = counted(plain)
    ex["batched_pairs"] = len(pairs)
    ex["batched_points"] = int(sum(b.x.shape[0] + b.z.shape[0] for b in pairs))
    ex["batched_registrations_per_s"] = len(pairs) / tb
    ex["plain_loop_registrations_per_s"] = len(pairs) / tp
    ex["batched_counts"] = cb
    ex["plain_loop_counts"] = cp
    # autotune the density classes on representative pairs of each shape
    # (stereo: dense, middle and sparse lengthscales; RGB-D: 0.1 and 0.05)
    t0 = time.perf_counter()
    for q, ells in ((next(b for b in pairs if "stereo" in b.name), (0.95, 0.3, 0.12)),
                    (next(b for b in pairs if "rgbd" in b.name), (0.1, 0.05))):
        X, Z, U, V = (torch.from_numpy(a).to(dev) for a in (q.x, q.z, q.u, q.v))
        for ell in ells:
            cvo.cvo_autotune(X, Z, q.T_gt, ell, U, V, spec)
    ex["autotune_s"] = time.perf_counter() - t0
    tbt, cbt = counted(batched)
    tpt, cpt = counted(plain)
    ex["batched_autotuned_registrations_per_s"] = len(pairs) / tbt
    ex["plain_loop_autotuned_registrations_per_s"] = len(pairs) / tpt
    ex["batched_autotuned_counts"] = cbt
    cvo.cvo_clear_tuning()
    # backward form: stereo-shaped pairs of 10k points, 32-dim LIN features
    lb = synth.learned_batch(seed=1003, batch=2)
    tot = 0.0
    for q in lb:
        X, Z, U, V = (torch.from_numpy(a).to(dev) for a in (q.x, q.z, q.u, q.v))
        sec, _ = timed(lambda: (cvo.cvo_inner_product(X, Z, q.T_eval, q.ell, U, V, q.spec),
                                cvo.cvo_inner_product_backward(X, Z, q.T_eval, q.ell, 1.0, U, V, q.spec)), 3)
        tot += sec
    ex["forward_backward_ms_per_pair_10k_lin32"] = 1e3 * tot / len(lb)
    # frame-to-frame odometry: 8 stereo frames of 30k points (7 pairs), the
    # first from the identity (0.95 -> 0.1), later ones warm-started at 0.1
    s = synth.stereo_sequence(frames=8)
    fr = [(torch.from_numpy(x).to(dev), torch.from_numpy(u).to(dev)) for x, u in s.frames]
    sec, (Ts, reps) = timed(lambda: cvo.cvo_odometry(fr, s.spec, s.first, s.rest), 1)
    dt, dr = s.drift(list(Ts))
    ex["odometry_pairs"] = len(Ts)
    ex["odometry_ms"] = 1e3 * sec
    ex["odometry_registrations_per_s"] = len(Ts) / sec
    ex["odometry_warm_iterations_mean"] = float(np.mean([r["iterations"] for r in reps[1:]]))
    ex["odometry_drift_pct"] = dt
    ex["odometry_drift_deg_per_m"] = dr
    # point selection on full 1241 x 376 stereo frames (24 feature channels),
    # at most 15000 points, then registration of the two selected clouds
    s = synth.stereo_images(frames=2)
    imgs = [tuple(torch.from_numpy(a).to(dev) for a in (f.gray, f.depth, f.feat)) for f in s.frames]
    sec, (xyz, fo, th, _) = timed(lambda: cvo.cvo_select_points(*imgs[0], s.camera, 15000), 20)
    ex["select_ms_per_frame"] = 1e3 * sec
    ex["select_points"] = int(xyz.shape[0])
    ex["select_threshold"] = th
    sel = [cvo.cvo_select_points(*im, s.camera, 15000)[:2] for im in imgs]
    prm = dict(ell_init=0.95, ell_min=0.1, max_iter=4000)
    sec, (T, rep, _) = timed(lambda: cvo.cvo_align(sel[0][0], sel[1][0], sel[0][1], sel[1][1], s.spec, prm), 3)
    R = np.linalg.inv(s.relative(0)) @ T
    ex["selected_registration_ms"] = 1e3 * sec
    ex["selected_registration_rot_err_deg"] = float(np.degrees(np.arccos(np.clip((np.trace(R[:3, :3]) - 1) / 2, -1, 1))))
    ex["selected_registration_trans_err_m"] = float(np.linalg.norm(R[:3, 3]))
    # the paper's pipeline on 8 image frames: select 3k-15k points per frame,
    # then frame-to-frame registration (first pair 0.95 -> 0.1, then 0.1)
    s = synth.stereo_images(frames=8)
    imgs = [tuple(torch.from_numpy(a).to(dev) for a in (f.gray, f.depth, f.feat)) for f in s.frames]
    first, rest = dict(ell_init=0.95, ell_min=0.1, max_iter=4000), dict(ell_init=0.1, ell_min=0.1, max_iter=4000)

    def pipeline():
        sel = [cvo.cvo_select_points(*im, s.camera, 15000)[:2] for im in imgs]
        return cvo.cvo_odometry(sel, s.spec, first, rest)

    sec, (Ts, reps) = timed(pipeline, 1)
    dt, dr = synth.trajectory_drift(s.poses, list(Ts))
    ex["selected_odometry_frames"] = len(imgs)
    ex["selected_odometry_ms"] = 1e3 * sec
    ex["selected_odometry_drift_pct"] = dt
    ex["selected_odometry_drift_deg_per_m"] = dr
    return ex


if __name__ == "__main__":
    main()
