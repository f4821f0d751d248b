"""Benchmark of the gradient-guided Monte Carlo SLAM filter step on one MI355X.

Workload (corridors): N = 100,000 particles, M = 2,048 points per scan (32 rings
x 64 azimuths, range <= 60 m), a 512 x 512 x 128 FP32 likelihood grid at 0.2 m
over a procedural corridor maze, a seeded 200-frame trajectory.  One step is
one frame: prediction with odometry and per-particle noise, 3 passes of
likelihood + gradient + pose step, weighting, log-sum-exp/ESS, and systematic
resampling when ESS < N/2.  Scans, noise and the map are resident in HBM
before timing starts.

Prints one JSON line with the particle x point evaluation rate (N * M * passes
per step / time), ms per step, the roofline of the dominant kernel (timed live
with HIP events on the session's stream) and the FP64 CPU oracle timed on the
host's cores on one frame.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle×point lik+grad evals/s; ms/step @100k particles; p99 session ms"
HBM_PEAK_GBS = 8000.0
BYTES_PER_EVAL = {0: 32, 1: 16, 2: 16}    # 8 grid samples per evaluation


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def run_cpu_baseline(c, frame, n_sample):
    """The FP64 oracle on one frame for n_sample particles, all host threads."""
    import oracle
    from synth import configs
    N = n_sample
    poses = c["poses"][:N]
    p = dict(c["params"])
    noise = configs.prediction_noise(N, frame, c["noise_sigma"], c["noise_seed"])
    t0 = time.perf_counter()
    oracle.filter_step(c["grid"], c["dims"], c["origin"], c["h"], c["scans"][frame], poses,
                       np.full(N, -math.log(N)), p, float(c["u"][frame]), policy=2,
                       ess_frac=p["ess_frac"], dT=c["odometry"][frame].astype(np.float64),
                       delta=noise, nthreads=cpu_cores())
    dt = time.perf_counter() - t0
    evals = N * c["scans"].shape[1] * p["iters"]
    return evals / dt, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--particles", type=int, default=100000)
    ap.add_argument("--grid-dtype", type=int, default=0, help="0 FP32, 1 FP16, 2 BF16")
    ap.add_argument("--cpu-sample", type=int, default=100000,
                    help="particles in the one-frame oracle timing (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2504_18056_amd import abi
    from synth import configs

    N = args.particles
    n_frames = 200
    t0 = time.perf_counter()
    c = configs.corridors(N=N, n_frames=n_frames, grid_dtype=args.grid_dtype)
    M = c["scans"].shape[1]
    log("inputs: corridors N=%d M=%d grid=%s (%.1f s)" % (N, M, c["dims"], time.perf_counter() - t0))

    dev = torch.device("cuda:0")
    scans = torch.from_numpy(np.ascontiguousarray(c["scans"])).to(dev)
    n_need = args.warmup + args.steps
    frames = [1 + (k % (n_frames - 1)) for k in range(n_need)]
    uniq = sorted(set(frames))
    noise_host = np.stack([configs.prediction_noise(N, f, c["noise_sigma"], c["noise_seed"])
                           for f in uniq])
    noise = torch.from_numpy(noise_host).to(dev)
    slot = {f: k for k, f in enumerate(uniq)}
    log("noise for %d frames uploaded (%.1f MB)" % (len(uniq), noise_host.nbytes / 1e6))

    ctx = abi.mcs_create(0)
    mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"], args.grid_dtype),
                           c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M)
    stream = abi.mcs_session_stream(ctx, sid)
    base = dict(c["params"], resample=abi.RESAMPLE_ESS, ess_frac=0.5)

    def step(f):
        p = dict(base, u=float(c["u"][f]), delta_T=c["odometry"][f])
        abi.mcs_filter_step_dev(ctx, sid, scans[f].data_ptr(), M, p,
                                noise_dev_ptr=noise[slot[f]].data_ptr(), stream=stream)

    for k in range(args.warmup):
        step(frames[k])
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    abi.mcs_session_profile(ctx, sid, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, n_need):
        step(frames[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = abi.mcs_session_profile_read(ctx, sid)
    abi.mcs_session_profile(ctx, sid, False)
    out = abi.mcs_get_particles(ctx, sid, N, poses=True, logw=False, parents=False, loglik=False,
                                grad=False)
    best = out["stats"]["best_pose"]
    f_last = frames[-1]
    err = float(np.linalg.norm(best[:3] - c["t_traj"][f_last]))
    log("timed %d steps: %.3f ms/step; eval %.3f ms/step; representative error %.3f m" % (
        args.steps, 1e3 * wall / args.steps, prof["eval_ms"] / max(1, prof["steps"]), err))
    abi.mcs_destroy(ctx)

    passes = base["iters"]
    evals_per_step = N * M * passes
    value = evals_per_step * args.steps / wall
    eval_s = prof["eval_ms"] * 1e-3 / max(1, prof["steps"])   # one eval launch per step
    bpe = BYTES_PER_EVAL[args.grid_dtype]
    achieved = bpe * evals_per_step / eval_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    stage_ms = {k: round(prof[k] / max(1, prof["steps"]), 4)
                for k in ("predict_ms", "eval_ms", "weights_ms", "resample_ms")}

    cpu = None
    if args.cpu_sample > 0:
        ns = min(args.cpu_sample, N)
        log("cpu baseline: oracle on frame 1, %d particles, %d threads" % (ns, cpu_cores()))
        rate, dt = run_cpu_baseline(c, 1, ns)
        cpu = {"value": round(rate, 1), "unit": "particle×point evals/s", "cores": cpu_cores(),
               "kind": "oracle",
               "sample": "one corridors frame (prediction, 3 passes, weights, ESS resampling) "
                         "for %d particles x %d points; %.2f s wall" % (ns, M, dt)}

    dtype_name = {0: "fp32", 1: "fp32 (fp16 grid)", 2: "fp32 (bf16 grid)"}[args.grid_dtype]
    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "particle×point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {"workload": "corridors: N=%d particles, M=%d points, 512x512x128 grid at 0.2 m, "
                               "3 gradient passes/frame, resample when ESS<N/2" % (N, M),
                   "particles": N, "points": M, "passes": passes,
                   "grid": list(c["dims"]), "grid_dtype": dtype_name},
        "stage_ms": stage_ms,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
