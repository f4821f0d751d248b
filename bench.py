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
# Algorithmic arithmetic of one (particle, point) evaluation, in FLOPs with an
# FMA counted as two (the method's operations, independent of how the kernel
# compiles them): transform u = A p + b, 9 FMA (18); cell index and fraction,
# 3 floor + 3 subtract (6); trilinear value and gradient from the cell's 8
# polynomial coefficients, 13 FMA + 3 multiplies (29); G + eps, ln, reciprocal
# (3); gradient scale, 3 multiplies (3); accumulation of l, sum d and
# sum v x d: 1 + 3 adds, cross product 3 multiplies + 3 FMA, 3 adds (16).
FLOPS_PER_EVAL = 75
# Published MI355X vector FP32 rate (256 CU x 2.4 GHz; an FMA = 2 FLOPs).
FP32_PEAK_TFLOPS = 157.3
BYTES_PER_EVAL = {0: 32, 1: 16, 2: 16}    # one cell record per evaluation
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_eval_corridors_100k_counters.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2504_18056_amd", "csrc", "kernels.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def counter_summary(grid_dtype):
    """The committed counter summary of the evaluation stage as a dict of its
    "key: value" lines, or None when it is missing, is for another grid dtype,
    or was taken on a different kernel source."""
    import hashlib
    try:
        with open(PMC_SUMMARY) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if kv.get("kernel_source_sha256", "").strip() != sha or int(kv.get("grid_dtype", -1)) != grid_dtype:
        return None
    return kv


def measured_traffic(grid_dtype):
    """HBM bytes per launch of the evaluation kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings), or
    None (see counter_summary)."""
    kv = counter_summary(grid_dtype)
    return None if kv is None else float(kv["hbm_bytes_per_launch"])


def issue_ceilings(rates, evals_per_s, grid_dtype):
    """VALU issue ceiling of the evaluation stage from the measured per-class
    issue rates (mcs_measure_issue_rates) and the stage's instruction mix per
    evaluation (SQ_INSTS_VALU_* counters of the committed summary): every
    instruction issued at its own class's measured rate, one after another,
    1 / sum_c (n_c / rate_c) evaluations per second."""
    kv = counter_summary(grid_dtype)
    if kv is None or rates is None:
        return None
    per = lambda k: float(kv[k].split()[0])
    total = per("valu_lane_ops_per_eval")
    mix = {"fp32": per("sq_insts_valu_fma_f32_per_eval") + per("sq_insts_valu_mul_f32_per_eval") +
                   per("sq_insts_valu_add_f32_per_eval"),
           "fp64": per("sq_insts_valu_fma_f64_per_eval") + per("sq_insts_valu_add_f64_per_eval"),
           "cvt": per("sq_insts_valu_cvt_per_eval"),
           "int32": per("sq_insts_valu_int32_per_eval"),
           "trans": per("sq_insts_valu_trans_f32_per_eval")}
    mix["other"] = max(0.0, total - sum(mix.values()))
    rate_of = {"fp32": rates["fp32_fma"], "fp64": rates["fp64_fma"], "cvt": rates["fp64_unary"],
               "int32": rates["int24"], "trans": rates["trans"], "other": rates["int24"]}
    by_class = 1.0 / sum(mix[k] / rate_of[k] for k in mix)
    return {"rates_T_lane_ops_per_s": {k: round(v / 1e12, 2) for k, v in rates.items()},
            "valu_per_eval": round(total, 2), "mix_per_eval": {k: round(v, 2) for k, v in mix.items()},
            "ceiling_evals_per_s": round(by_class, 1),
            "evals_per_s": round(evals_per_s, 1),
            "frac": round(evals_per_s / by_class, 4),
            "note": "rates: eight independent chains per lane of one instruction class over the "
                    "whole device (fp32: v_fmac_f32; fp64: v_fmac_f64; fp64_unary: v_fract_f64, "
                    "the class of floor and FP64 conversions; int24: v_mad_u32_u24; trans: "
                    "v_rcp_f32; fp32_fp64: v_fmac_f32 and v_fmac_f64 alternating); mix: the evaluation stage's VALU instructions per evaluation "
                    "by class from %s (other: the rest, at the int24 rate)"
                    % os.path.relpath(PMC_SUMMARY, ROOT)}


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def device_copy_gbps(torch, mib=1024, reps=10):
    """HBM bandwidth of a plain device-to-device copy (bytes read + written per
    second), the stream-copy figure beside the evaluation's gather rate."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    secs = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 2.0 * n * 4 / secs / 1e9


def eval_vs_floor(abi, torch, ctx, sid, scan_dev, M, p, poses, logw, reps=10):
    """Evaluation stage against its gather floor from one state: `reps` times
    the likelihood passes of a step (no prediction, no resampling) and `reps`
    times the gather-floor passes (same tiling, transformed coordinates and
    record loads; a checksum instead of the arithmetic), each restarted from
    the same poses.  Mean stage times from the library's HIP events."""
    q = dict(p, resample=abi.RESAMPLE_NEVER, beta=0.0)
    q.pop("delta_T", None)
    out = {}
    for name in ("eval", "floor"):
        total, steps = 0.0, 0
        for _ in range(reps):
            abi.mcs_set_particles(ctx, sid, poses=poses, logw=logw)
            abi.mcs_session_profile(ctx, sid, True)
            if name == "eval":
                abi.mcs_filter_step_dev(ctx, sid, scan_dev, M, q)
            else:
                abi.mcs_gather_floor_dev(ctx, sid, scan_dev, M, q)
            pr = abi.mcs_session_profile_read(ctx, sid)
            abi.mcs_session_profile(ctx, sid, False)
            total += pr["eval_ms"]
            steps += pr["steps"]
        out[name + "_ms"] = round(total / max(1, steps), 4)
    out["frac_of_floor_rate"] = round(out["floor_ms"] / out["eval_ms"], 4)
    return out


def run_trajectory(abi, torch, ctx, mid, c, base):
    """The whole seeded trajectory from the initial spread, one step per frame
    (the benchmark's step: prediction with odometry and per-particle noise, 3
    passes, ESS resampling); per frame the representative's (max-weight
    particle's) translation and rotation error against the true pose."""
    from scipy.spatial.transform import Rotation
    from synth import configs
    N = c["poses"].shape[0]
    M = c["scans"].shape[1]
    n = c["scans"].shape[0]
    dev = torch.device("cuda:0")
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M)
    terr, rerr, ess, res = [], [], [], 0
    try:
        scans = torch.from_numpy(np.ascontiguousarray(c["scans"])).to(dev)
        for f in range(1, n):
            noise = torch.from_numpy(configs.prediction_noise(N, f, c["noise_sigma"], c["noise_seed"])).to(dev)
            p = dict(base, u=float(c["u"][f]), delta_T=c["odometry"][f])
            abi.mcs_filter_step_dev(ctx, sid, scans[f].data_ptr(), M, p, noise_dev_ptr=noise.data_ptr())
            st = abi.mcs_get_particles(ctx, sid, poses=False, logw=False, parents=False, loglik=False,
                                       grad=False)["stats"]
            b = st["best_pose"].astype(np.float64)
            terr.append(float(np.linalg.norm(b[:3] - c["t_traj"][f])))
            qt = np.asarray(c["q_traj"][f], np.float64)
            rel = Rotation.from_quat([qt[1], qt[2], qt[3], qt[0]]).inv() * \
                Rotation.from_quat([b[4], b[5], b[6], b[3]])
            rerr.append(float(np.degrees(rel.magnitude())))
            ess.append(st["ess"])
            res += int(st["resampled"])
    finally:
        abi.mcs_session_destroy(ctx, sid)
    t, r = np.array(terr), np.array(rerr)
    return {"frames": n - 1, "representative_translation_error_m":
            {"mean": round(float(t.mean()), 4), "median": round(float(np.median(t)), 4),
             "p95": round(float(np.percentile(t, 95)), 4), "max": round(float(t.max()), 4),
             "final": round(float(t[-1]), 4)},
            "representative_rotation_error_deg":
            {"mean": round(float(r.mean()), 3), "median": round(float(np.median(r)), 3),
             "max": round(float(r.max()), 3), "final": round(float(r[-1]), 3)},
            "resampled_frames": res, "ess_median": round(float(np.median(ess)), 1)}


def run_cpu_baseline(c, frame, n_sample, threads=None):
    """The FP64 oracle on one frame for n_sample particles (all host threads by default)."""
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
                       delta=noise, nthreads=threads or cpu_cores())
    dt = time.perf_counter() - t0
    evals = N * c["scans"].shape[1] * p["iters"]
    return evals / dt, dt


def _session_inputs(desc):
    from synth import configs
    x = configs.serving_session_inputs(desc)
    x["grid"] = np.ascontiguousarray(x["grid"])
    return desc, x


def prepare_serving(args):
    """Inputs of the serving sessions, built by worker processes before the GPU is touched."""
    from concurrent.futures import ProcessPoolExecutor

    from synth import configs
    descs = configs.serving_sessions(n_sessions=args.serving_sessions, n_scans=4)
    t0 = time.perf_counter()
    workers = max(1, min(8, cpu_cores() // 2))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        out = list(ex.map(_session_inputs, descs))
    log("serving inputs: %d sessions built in %.1f s" % (len(out), time.perf_counter() - t0))
    return out


def run_serving(args, abi, torch, prepared, load=None, seconds=None, admission=True):
    """Many concurrent sessions with Poisson frame arrivals: batched server vs one at a time.
    load multiplies the 10 Hz per-session arrival rate; seconds is the schedule's length."""
    load = args.serving_load if load is None else load
    seconds = args.serving_seconds if seconds is None else seconds
    from synth import configs
    dev = torch.device("cuda:0")
    ctx = abi.mcs_create(0)
    sessions = []
    t0 = time.perf_counter()
    for desc, x in prepared:
        mid = abi.mcs_init_map(ctx, abi.grid_desc(x["dims"], x["origin"], x["h"], abi.GRID_FP16),
                               x["grid"])
        N, M = desc["N"], desc["M"]
        sid = abi.mcs_session_create(ctx, mid, x["poses"], M_max=M)
        rng = np.random.default_rng(desc["seed"] + 9)
        noise = (rng.normal(size=(x["scans"].shape[0], N, 6)) *
                 [0.05, 0.05, 0.05, 0.017, 0.017, 0.017]).astype(np.float32)
        sessions.append(dict(desc=desc, sid=sid, mid=mid, N=N, M=M, poses=x["poses"],
                             params=x["params"], odo=x["odometry"], u=x["u"],
                             scans=torch.from_numpy(x["scans"]).to(dev),
                             noise=torch.from_numpy(noise).to(dev)))
    torch.cuda.synchronize()
    mem = abi.mcs_memory_in_use(ctx)
    log("serving: %d sessions ready (%.1f s), %.2f GB resident, N mean %.0f, M mean %.0f" % (
        len(sessions), time.perf_counter() - t0, mem / 1e9,
        np.mean([s["N"] for s in sessions]), np.mean([s["M"] for s in sessions])))

    rng = np.random.default_rng(4242)
    arrivals = []
    for k, s in enumerate(sessions):
        for t in configs.poisson_arrivals(10.0 * load, seconds, rng):
            arrivals.append((t, k))
    arrivals.sort()
    results = {}
    modes = ((abi.SERVE_BATCHED, "batched"), (abi.SERVE_CONCURRENT, "concurrent"),
             (abi.SERVE_SERIAL, "one_at_a_time"))
    for mode, name in modes:
        for s in sessions:
            abi.mcs_set_particles(ctx, s["sid"], poses=s["poses"], logw=np.full(s["N"], -math.log(s["N"])))
        torch.cuda.synchronize()
        srv = abi.mcs_server_create(ctx, mode=mode, dtype=abi.GRID_FP16, max_batch=len(sessions))
        counts = [0] * len(sessions)
        ids = []
        start = time.perf_counter()
        for t, k in arrivals:
            delay = start + t - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            s = sessions[k]
            f = counts[k] % s["scans"].shape[0]
            p = dict(s["params"], u=float(s["u"][counts[k] % len(s["u"])]), resample=abi.RESAMPLE_ESS,
                     delta_T=s["odo"][f])
            counts[k] += 1
            ids.append(abi.mcs_server_submit(srv, s["sid"], s["scans"][f].data_ptr(), s["M"], p,
                                             noise_dev_ptr=s["noise"][f].data_ptr()))
        abi.mcs_server_drain(srv)
        times = [abi.mcs_server_times(srv, r) for r in ids]
        st = abi.mcs_server_stats_get(srv)
        abi.mcs_server_destroy(srv)
        lat = np.array([(t["done_ns"] - t["submit_ns"]) * 1e-6 for t in times])
        wait = np.array([(t["launch_ns"] - t["submit_ns"]) * 1e-6 for t in times])
        run = np.array([(t["done_ns"] - t["launch_ns"]) * 1e-6 for t in times])
        span = (max(t["done_ns"] for t in times) - min(t["submit_ns"] for t in times)) * 1e-9
        pct = lambda a, q: round(float(np.percentile(a, q)), 3)
        results[name] = {"p50_ms": pct(lat, 50), "p90_ms": pct(lat, 90), "p99_ms": pct(lat, 99),
                         "mean_ms": round(float(lat.mean()), 3),
                         "queue_p50_ms": pct(wait, 50), "queue_p99_ms": pct(wait, 99),
                         "run_p50_ms": pct(run, 50), "run_p99_ms": pct(run, 99),
                         "frames": len(ids), "launches": st["ticks"],
                         "max_in_flight": st["max_batch_seen"],
                         "evals_per_s": round(st["evals"] / span, 1)}
        log("serving %s: %s" % (name, results[name]))
    abi.mcs_destroy(ctx)
    if not admission:
        return {"sessions": len(sessions), "seconds": seconds, "arrival_hz_per_session": 10.0 * load,
                "offered_frames_per_s": round(len(arrivals) / seconds, 1),
                "resident_gb": round(mem / 1e9, 2), **results}
    # Admission under an HBM budget of half the footprint: sessions are admitted
    # in order until the next one would exceed the budget.
    budget = mem // 2
    actx = abi.mcs_create(0, hbm_budget_bytes=budget)
    admitted = refused = 0
    for desc, x in prepared:
        try:
            mid = abi.mcs_init_map(actx, abi.grid_desc(x["dims"], x["origin"], x["h"], abi.GRID_FP16),
                                   x["grid"])
        except abi.McsError as e:
            if e.status != abi.MCS_EBUDGET:
                raise
            refused += 1
            continue
        try:
            abi.mcs_session_create(actx, mid, x["poses"], M_max=desc["M"])
            admitted += 1
        except abi.McsError as e:
            if e.status != abi.MCS_EBUDGET:
                raise
            abi.mcs_release_map(actx, mid)
            refused += 1
    in_use = abi.mcs_memory_in_use(actx)
    abi.mcs_destroy(actx)
    return {"sessions": len(sessions), "seconds": seconds,
            "arrival_hz_per_session": 10.0 * load,
            "offered_frames_per_s": round(len(arrivals) / seconds, 1),
            "resident_gb": round(mem / 1e9, 2), **results,
            "admission_at_half_budget": {"budget_gb": round(budget / 1e9, 2), "admitted": admitted,
                                         "refused": refused, "in_use_gb": round(in_use / 1e9, 2)}}


def run_gicp(abi, steps=5):
    """GICP likelihood with Gauss-Newton passes: K = 64 voxel keyframe maps (64^3
    voxels of 0.4 m), N = 50,000, M = 2,048, 4 neighbours, 3 passes."""
    import torch
    from synth import configs
    c = configs.keyframes(N=50000, K=64, gicp=True)
    K = c["vox"].shape[0]
    ctx = abi.mcs_create(0)
    descs = [abi.voxel_desc(c["vox_dims"], c["vox_origins"][k], c["vox_edge"]) for k in range(K)]
    mid = abi.mcs_load_gicp_keyframes(ctx, descs, [c["vox"][k] for k in range(K)])
    N, M = c["poses"].shape[0], c["scan"].shape[0]
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M, kf_poses=c["kf_poses"])
    mu = torch.from_numpy(c["scan"]).to("cuda:0")
    cov = torch.from_numpy(c["scan_cov"]).to("cuda:0")
    p = dict(c["params"], iters=3, u=c["u"], beta=0.001, resample=abi.RESAMPLE_ESS)
    abi.mcs_filter_step_gicp_dev(ctx, sid, mu.data_ptr(), cov.data_ptr(), M, p)
    torch.cuda.synchronize()
    abi.mcs_session_profile(ctx, sid, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        abi.mcs_filter_step_gicp_dev(ctx, sid, mu.data_ptr(), cov.data_ptr(), M, p)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = abi.mcs_session_profile_read(ctx, sid)
    abi.mcs_destroy(ctx)
    evals = N * M * 3 * p["n_neighbors"]
    return {"workload": "GICP keyframes: K=64 maps of 64^3 voxels at 0.4 m, N=50000, M=2048, "
                        "4 neighbours, 3 Gauss-Newton passes",
            "ms_per_step": round(1e3 * wall / steps, 3),
            "eval_ms_per_step": round(prof["eval_ms"] / max(1, prof["steps"]), 3),
            "evals_per_s": round(evals * steps / wall, 1),
            "note": "an evaluation is one (particle, point, neighbour) voxel lookup, residual, "
                    "3x3 inverse and 28-term accumulation"}


FLOORS_NOISE_SIGMA = (0.03, 0.03, 0.005, 0.002, 0.002, 0.008)


def floors_run(c, policy, beta=0.05, ctx=None):
    """Kidnapped start over identical storeys, run through the library: each frame
    prediction with odometry and device-drawn random-walk noise, gradient passes,
    weighting and dead-particle pruning (or ESS resampling).  Returns the
    per-frame share of the weight mass and of the particles on each storey, and
    the representative's storey."""
    from paper_2504_18056_amd import abi
    own = ctx is None
    ctx = abi.mcs_create(0) if own else ctx
    N = c["poses"].shape[0]
    M = c["scans"].shape[1]
    mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M)
    z0 = c["t_traj"][0][2] - c["true_floor"] * c["storey"]
    mass, share, best = [], [], []
    try:
        for f in range(c["scans"].shape[0]):
            p = dict(c["params"], u=float(c["u"][f]), beta=beta, resample=policy, ess_frac=0.5,
                     prune_post=1e-8, prune_lik=1e-16, noise_mode=abi.NOISE_DEVICE, rng_seed=77,
                     rng_frame=f, noise_sigma=FLOORS_NOISE_SIGMA)
            if f > 0:
                p["delta_T"] = c["odometry"][f]
            abi.mcs_filter_step(ctx, sid, c["scans"][f], p)
            o = abi.mcs_get_particles(ctx, sid, N, parents=False, loglik=False, grad=False)
            fl = np.clip(np.rint((o["poses"][:, 2] - z0) / c["storey"]), 0, c["floors"] - 1).astype(int)
            w = np.exp(o["logw"])
            mass.append(np.bincount(fl, weights=w, minlength=c["floors"]) / w.sum())
            share.append(np.bincount(fl, minlength=c["floors"]) / N)
            bz = o["stats"]["best_pose"][2]
            best.append(int(np.clip(round((bz - z0) / c["storey"]), 0, c["floors"] - 1)))
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)
        if own:
            abi.mcs_destroy(ctx)
    return np.array(mass), np.array(share), np.array(best)


def floors_summary(c, mass, share, best):
    """Storey shares before the distinguishing feature is seen, and convergence after."""
    t = c["true_floor"]
    fs = c["first_seen"]
    conv = [f for f in range(fs, len(mass)) if mass[f, t] > 0.9]
    return {"first_seen_frame": int(fs),
            "floors_with_5pct_particles_before": int(np.sum(share[fs - 1] >= 0.05)),
            "mass_per_floor_before": [round(float(x), 3) for x in mass[fs - 1]],
            "true_floor_mass_end": round(float(mass[-1, t]), 4),
            "frames_to_90pct_after_first_seen": (conv[0] - fs) if conv else None,
            "representative_on_true_floor_end": bool(best[-1] == t)}


def run_floors(abi):
    """Kidnapped start over four identical storeys (N = 20,000, 80 frames): storey
    shares before the distinguishing feature is seen, and convergence after."""
    from synth import configs
    c = configs.repeated_floors(N=20000)
    out = {"workload": "repeated floors: 4 identical storeys of a 51.2 m maze level, one box only on "
                       "the true storey, N=20000, M=512, 10 m range, 80 frames, beta=0.05, "
                       "device random-walk noise"}
    for policy, name in ((abi.RESAMPLE_PRUNE, "pruning"), (abi.RESAMPLE_ESS, "ess_resampling")):
        t0 = time.perf_counter()
        mass, share, best = floors_run(c, policy)
        out[name] = dict(floors_summary(c, mass, share, best),
                         ms_per_frame=round(1e3 * (time.perf_counter() - t0) / len(mass), 3))
    return out


def run_keyframes(abi, steps=5):
    """Keyframe-map step timing: K = 64 grids, N = 50,000, M = 2,048, 4 neighbours, 3 passes,
    on a path that returns to its start, with the keyframes fixed and with the loop-gated
    correction that propagates each step along the particle's keyframes."""
    import torch
    from synth import configs
    c = configs.keyframes(N=50000, K=64, out_and_back=True)
    K = c["grids"].shape[0]
    ctx = abi.mcs_create(0)
    descs = [abi.grid_desc(c["dims"], c["origins"][k], c["h"]) for k in range(K)]
    mid = abi.mcs_load_keyframes(ctx, descs, [c["grids"][k] for k in range(K)])
    N, M = c["poses"].shape[0], c["scan"].shape[0]
    scan = torch.from_numpy(c["scan"]).to("cuda:0")
    res = {"workload": "keyframes: K=64 local 128^3 grids, N=50000, M=2048, 4 neighbours, "
                       "3 passes, out-and-back path (the current frame revisits the first keyframes)",
           "note": "an evaluation is one (particle, point, neighbour) trilinear sample"}
    for mode, name in ((abi.KF_FIXED, "fixed_keyframes"), (abi.KF_LOOP, "loop_update")):
        sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M, kf_poses=c["kf_poses"])
        p = dict(c["params"], iters=3, u=c["u"], resample=abi.RESAMPLE_ESS, kf_update=mode)
        abi.mcs_filter_step_dev(ctx, sid, scan.data_ptr(), M, p)
        torch.cuda.synchronize()
        abi.mcs_session_profile(ctx, sid, True)
        t0 = time.perf_counter()
        for _ in range(steps):
            abi.mcs_filter_step_dev(ctx, sid, scan.data_ptr(), M, p)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = abi.mcs_session_profile_read(ctx, sid)
        abi.mcs_session_destroy(ctx, sid)
        evals = N * M * 3 * p["n_neighbors"]
        res[name] = {"ms_per_step": round(1e3 * wall / steps, 3),
                     "eval_ms_per_step": round(prof["eval_ms"] / max(1, prof["steps"]), 3),
                     "evals_per_s": round(evals * steps / wall, 1),
                     "grid_element_gathers_per_s": round(8 * evals * steps / wall, 1)}
    abi.mcs_destroy(ctx)
    return res


def run_precision(abi, torch, c, scans, noise, slot, frames, base, steps=30, warm=5):
    """FP16 and BF16 grid records (corridors, the same frames): ms per step, the
    evaluation stage, and the log-likelihoods of the first frame against the
    FP32 records' (the quantisation error of the stored grid, stated)."""
    N, M = c["poses"].shape[0], c["scans"].shape[1]
    out, l32 = {}, None
    for dt, name in ((0, "fp32"), (1, "fp16"), (2, "bf16")):
        ctx = abi.mcs_create(0)
        mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"], dt), c["grid"])
        sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M)

        def step(f, resample=abi.RESAMPLE_ESS):
            p = dict(base, u=float(c["u"][f]), delta_T=c["odometry"][f], resample=resample)
            abi.mcs_filter_step_dev(ctx, sid, scans[f].data_ptr(), M, p,
                                    noise_dev_ptr=noise[slot[f]].data_ptr())

        step(frames[0], abi.RESAMPLE_NEVER)
        l = abi.mcs_get_particles(ctx, sid, N)["loglik"].astype(np.float64)
        abi.mcs_set_particles(ctx, sid, poses=c["poses"], logw=np.full(N, -math.log(N)))
        for k in range(warm):
            step(frames[k % len(frames)])
        torch.cuda.synchronize()
        abi.mcs_session_profile(ctx, sid, True)
        t0 = time.perf_counter()
        for k in range(warm, warm + steps):
            step(frames[k % len(frames)])
        abi.mcs_session_sync(ctx, sid)
        wall = time.perf_counter() - t0
        prof = abi.mcs_session_profile_read(ctx, sid)
        abi.mcs_destroy(ctx)
        r = {"ms_per_step": round(1e3 * wall / steps, 4),
             "eval_ms": round(prof["eval_ms"] / max(1, prof["steps"]), 4),
             "evals_per_s": round(N * M * base["iters"] * steps / wall, 1)}
        if l32 is None:
            l32 = l
        else:
            rel = np.abs(l - l32) / np.abs(l32)
            r["loglik_rel_diff_vs_fp32_records"] = {"max": float("%.3g" % rel.max()),
                                                    "median": float("%.3g" % np.median(rel))}
        out[name] = r
    return {"workload": "corridors records in FP32, FP16 and BF16 (RNE from the FP32 grid): N=%d, "
                        "M=%d, 3 passes; first-frame log-likelihoods compared with the FP32 records'"
                        % (N, M), **out}


def run_ambiguous_rooms(abi):
    """Keyframe map of a row of identical rooms (translated copies), K = 64, N = 50,000,
    M = 2,048: the initial cloud copied at four room shifts (12,500 particles each), one step
    of 3 passes with beta = 0.01 and no resampling.  Reports the ESS, the weight held by each
    shift and the number of shifts holding at least 1 % of it (the translation modes)."""
    import torch
    from synth import configs
    c = configs.keyframes(N=50000, K=64, ambiguous=True)
    K = c["grids"].shape[0]
    room = c["scene"].rooms["room"]
    N, M = c["poses"].shape[0], c["scan"].shape[0]
    shift = np.repeat(np.arange(-2, 2), N // 4)
    poses = c["poses"].copy()
    poses[:, 0] += (shift * room).astype(np.float32)
    ctx = abi.mcs_create(0)
    descs = [abi.grid_desc(c["dims"], c["origins"][k], c["h"]) for k in range(K)]
    mid = abi.mcs_load_keyframes(ctx, descs, [c["grids"][k] for k in range(K)])
    sid = abi.mcs_session_create(ctx, mid, poses, M_max=M, kf_poses=c["kf_poses"])
    p = dict(c["params"], iters=3, u=0.5, beta=0.01, resample=abi.RESAMPLE_NEVER)
    t0 = time.perf_counter()
    abi.mcs_filter_step(ctx, sid, c["scan"], p)
    out = abi.mcs_get_particles(ctx, sid, N)
    wall = time.perf_counter() - t0
    abi.mcs_destroy(ctx)
    w = np.exp(out["logw"])
    mass = [float(w[shift == s].sum()) for s in range(-2, 2)]
    return {"workload": "keyframes over 6 identical rooms (8 m period): K=64, N=50000 as 4 copies "
                        "of the initial cloud shifted by -2..+1 rooms along the row, M=2048, "
                        "3 passes, beta=0.01",
            "ess": round(float(out["stats"]["ess"]), 3),
            "mass_per_room_shift": {str(s): round(m, 6) for s, m in zip(range(-2, 2), mass)},
            "modes_over_1pct": int(sum(m >= 0.01 for m in mass)),
            "step_ms_host_buffers": round(1e3 * wall, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--particles", type=int, default=100000)
    ap.add_argument("--grid-dtype", type=int, default=0, help="0 FP32, 1 FP16, 2 BF16")
    ap.add_argument("--cpu-sample", type=int, default=100000,
                    help="particles in the one-frame oracle timing (0: skip)")
    ap.add_argument("--serving-seconds", type=float, default=10.0,
                    help="length of the Poisson arrival schedule (0: skip serving)")
    ap.add_argument("--serving-sessions", type=int, default=64)
    ap.add_argument("--serving-load", type=float, default=1.0,
                    help="multiplier on the 10 Hz per-session arrival rate")
    ap.add_argument("--extras", type=int, default=1,
                    help="1: also report the record-precision table, the keyframe-map and GICP "
                         "timings and the repeated-floors demo; 2: only the keyframe-map and GICP "
                         "timings (for profiling those kernels)")
    ap.add_argument("--gather-floor", type=int, default=0,
                    help="only time the evaluation stage against its gather floor, this many "
                         "times each, from the cloud after the warm-up frames and from the "
                         "initial spread (for profiling those kernels)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe_mb > 0:
        import torch
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this implementation has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    prepared = prepare_serving(args) if args.serving_seconds > 0 else None
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

    # The first frame starts from the initial spread (0.5 m, 5 deg): the particles
    # touch far more cells than once converged, so it is timed on its own.
    abi.mcs_session_profile(ctx, sid, True)
    step(frames[0])
    torch.cuda.synchronize()
    first = abi.mcs_session_profile_read(ctx, sid)
    abi.mcs_session_profile(ctx, sid, False)
    first_eval_ms = first["eval_ms"] / max(1, first["steps"])
    log("first frame (initial spread): eval %.3f ms" % first_eval_ms)
    # The same frame from the same initial cloud again (the session ends in the
    # same state), now with the grid's pages and cache lines touched once: the
    # spread's own cost.
    abi.mcs_set_particles(ctx, sid, poses=c["poses"], logw=np.full(N, -math.log(N)))
    abi.mcs_session_profile(ctx, sid, True)
    step(frames[0])
    torch.cuda.synchronize()
    again = abi.mcs_session_profile_read(ctx, sid)
    abi.mcs_session_profile(ctx, sid, False)
    spread_eval_ms = again["eval_ms"] / max(1, again["steps"])
    log("initial spread, second time: eval %.3f ms" % spread_eval_ms)
    for k in range(1, args.warmup):
        step(frames[k])
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    if args.gather_floor > 0:
        st = abi.mcs_get_particles(ctx, sid, poses=True, logw=True, parents=False, loglik=False,
                                   grad=False, stats=False)
        f = frames[args.warmup - 1]
        pf = dict(base, u=float(c["u"][f]))
        res = {"workload": "corridors N=%d M=%d, %d passes" % (N, M, base["iters"]),
               "converged": eval_vs_floor(abi, torch, ctx, sid, scans[f].data_ptr(), M, pf,
                                          st["poses"], st["logw"], reps=args.gather_floor),
               "initial_spread": eval_vs_floor(abi, torch, ctx, sid, scans[frames[0]].data_ptr(), M, pf,
                                               c["poses"], np.full(N, -math.log(N)),
                                               reps=args.gather_floor)}
        abi.mcs_destroy(ctx)
        print(json.dumps(res), flush=True)
        return
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
    # Host-buffer entry point (scan and noise copied over PCIe each step), for reference.
    n_host = min(10, len(frames))
    scans_host = [np.ascontiguousarray(c["scans"][f]) for f in frames[:n_host]]
    noise_host_f = [noise_host[slot[f]] for f in frames[:n_host]]
    abi.mcs_session_sync(ctx, sid)
    t0 = time.perf_counter()
    for k in range(n_host):
        f = frames[k]
        abi.mcs_filter_step(ctx, sid, scans_host[k], dict(base, u=float(c["u"][f]), delta_T=c["odometry"][f]),
                            noise=noise_host_f[k])
    abi.mcs_session_sync(ctx, sid)
    host_ms = 1e3 * (time.perf_counter() - t0) / n_host
    log("host-buffer entry point: %.3f ms/step" % host_ms)
    # The evaluation stage against its gather floor (same tiling, coordinates
    # and record loads; the arithmetic cut to a checksum), from the converged
    # cloud of the last timed frame and from the initial spread.
    st = abi.mcs_get_particles(ctx, sid, poses=True, logw=True, parents=False, loglik=False,
                               grad=False, stats=False)
    pf = dict(base, u=float(c["u"][f_last]))
    floors_conv = eval_vs_floor(abi, torch, ctx, sid, scans[f_last].data_ptr(), M, pf,
                                st["poses"], st["logw"])
    floors_conv["state"] = "the cloud after the timed frames, frame %d's scan" % f_last
    floors_spread = eval_vs_floor(abi, torch, ctx, sid, scans[frames[0]].data_ptr(), M, pf,
                                  c["poses"], np.full(N, -math.log(N)))
    floors_spread["state"] = "the initial spread (0.5 m, 5 deg), frame %d's scan" % frames[0]
    log("gather floor: converged %s; initial spread %s" % (floors_conv, floors_spread))
    # The same scan visited ring by ring instead of in firing order: the
    # evaluation follows the given point order, whose locality reaches the caches.
    rings = 32
    ring_major = np.arange(M).reshape(M // rings, rings).T.reshape(-1)
    scan_rm = torch.from_numpy(np.ascontiguousarray(c["scans"][f_last][ring_major])).to(dev)
    rm = eval_vs_floor(abi, torch, ctx, sid, scan_rm.data_ptr(), M, pf, st["poses"], st["logw"])
    scan_order = {"firing_order_eval_ms": floors_conv["eval_ms"], "ring_major_eval_ms": rm["eval_ms"],
                  "note": "the converged cloud's evaluation stage with frame %d's points in the "
                          "sensor's firing order (every ring at one azimuth, then the next) and "
                          "ring by ring" % f_last}
    log("scan order: %s" % scan_order)
    trajectory = run_trajectory(abi, torch, ctx, mid, c, base)
    log("trajectory: %s" % trajectory)
    rates = abi.mcs_measure_issue_rates(ctx)
    log("VALU issue rates (T lane-ops/s): %s" % {k: round(v / 1e12, 2) for k, v in rates.items()})
    abi.mcs_destroy(ctx)
    copy_gbps = device_copy_gbps(torch)
    log("device copy: %.0f GB/s (read + write)" % copy_gbps)
    precision = None
    if args.extras == 1 and args.grid_dtype == 0:
        precision = run_precision(abi, torch, c, scans, noise, slot, frames, base)
        log("precision: %s" % precision)

    passes = base["iters"]
    evals_per_step = N * M * passes
    value = evals_per_step * args.steps / wall
    # The evaluation stage of a step: k_eval over the whole rounds of tiles and,
    # when the last round is small, the tail kernels beside it (HIP events on
    # the session stream around the stage).
    eval_s = prof["eval_ms"] * 1e-3 / max(1, prof["steps"])
    achieved = FLOPS_PER_EVAL * evals_per_step / eval_s / 1e12
    traffic = measured_traffic(args.grid_dtype)
    gbytes = BYTES_PER_EVAL[args.grid_dtype] * evals_per_step / 1e9
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": traffic,
                "kernel": "k_eval (with its tail kernels)", "eval_launch_ms": round(eval_s * 1e3, 4),
                "flops_per_eval": FLOPS_PER_EVAL,
                "gather_floor": floors_conv,
                "issue_ceiling": issue_ceilings(rates, evals_per_step / eval_s, args.grid_dtype),
                "gather_bytes_per_stage": round(gbytes * 1e9),
                "gather_rate_TBps": round(gbytes / eval_s / 1e3, 3),
                "note": "algorithmic FP32 arithmetic (%d FLOPs per evaluation, an FMA = 2) x %d "
                        "evaluations per step's evaluation stage / the stage's time, against the "
                        "published 157.3 TFLOP/s vector FP32 rate. gather_floor: the same passes "
                        "with the arithmetic cut to a checksum of the gathered records (same tiling, "
                        "coordinates and loads), timed from the same state; frac_of_floor_rate = "
                        "floor time / evaluation time. traffic = HBM bytes per stage from "
                        "FETCH_SIZE/WRITE_SIZE (%s); the algorithmic gather is %d B per evaluation, "
                        "served almost entirely from the caches"
                        % (FLOPS_PER_EVAL, evals_per_step, os.path.relpath(PMC_SUMMARY, ROOT),
                           BYTES_PER_EVAL[args.grid_dtype])}
    stage_ms = {k: round(prof[k] / max(1, prof["steps"]), 4)
                for k in ("predict_ms", "eval_ms", "weights_ms", "resample_ms")}

    cpu = cpu1 = None
    if args.cpu_sample > 0:
        ns = min(args.cpu_sample, N)
        log("cpu baseline: oracle on frame 1, %d particles, %d threads" % (ns, cpu_cores()))
        rate, dt = run_cpu_baseline(c, 1, ns)
        cpu = {"value": round(rate, 1), "unit": "particle×point evals/s", "cores": cpu_cores(),
               "kind": "oracle",
               "sample": "one corridors frame (prediction, 3 passes, weights, ESS resampling) "
                         "for %d particles x %d points; %.2f s wall" % (ns, M, dt)}
        n1 = max(1, ns // 50)
        rate1, dt1 = run_cpu_baseline(c, 1, n1, threads=1)
        cpu1 = {"value": round(rate1, 1), "unit": "particle×point evals/s", "cores": 1,
                "kind": "oracle",
                "sample": "the same frame for %d particles, one thread; %.2f s wall" % (n1, dt1)}

    floors = keyframes = gicp = None
    if args.extras:
        log("keyframe-map timing")
        keyframes = run_keyframes(abi)
        log("keyframes: %s" % keyframes)
        if args.extras == 1:
            keyframes["ambiguous_rooms"] = run_ambiguous_rooms(abi)
            log("ambiguous rooms: %s" % keyframes["ambiguous_rooms"])
        log("GICP timing")
        gicp = run_gicp(abi)
        log("gicp: %s" % gicp)
        if args.extras == 1:
            log("repeated-floors demo")
            floors = run_floors(abi)
            log("floors: %s" % floors)
    serving = None
    if args.serving_seconds > 0:
        serving = run_serving(args, abi, torch, prepared)
        # Three times the arrival rate, past what one-at-a-time execution
        # sustains: aggregate evaluations per second of each mode.
        serving["saturated"] = run_serving(args, abi, torch, prepared, load=3.0 * args.serving_load,
                                           seconds=max(1.0, args.serving_seconds / 2), admission=False)
        del prepared

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
        "gather_floor_initial_spread": floors_spread,
        "trajectory_200_frames": trajectory,
        "scan_order": scan_order,
        "eval_ms_first_frame_initial_spread": round(first_eval_ms, 4),
        "eval_ms_initial_spread_second_time": round(spread_eval_ms, 4),
        "trilinear_samples_per_s": round(value, 1),
        "grid_element_gathers_per_s": round(8 * value, 1),
        "host_buffers_ms_per_step": round(host_ms, 4),
        "device_copy_GBps": round(copy_gbps, 1),
        "hbm_equivalent_gather_evals_per_s": round(copy_gbps * 1e9 / BYTES_PER_EVAL[args.grid_dtype], 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_one_thread": cpu1,
        "ms_per_step_100k": round(1e3 * wall / args.steps, 4) if N == 100000 else None,
        "p99_session_ms": serving["batched"]["p99_ms"] if serving else None,
        "p99_session_ms_one_at_a_time": serving["one_at_a_time"]["p99_ms"] if serving else None,
        "serving": serving,
        "grid_record_precision": precision,
        "keyframes": keyframes,
        "gicp": gicp,
        "repeated_floors": floors,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
