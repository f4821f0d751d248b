"""Kidnapped start over identical storeys, run through the library (shared by
the GPU test and the benchmark's demo leg).  Each frame: prediction with
odometry and device-drawn random-walk noise, gradient passes, weighting, and
dead-particle pruning (or ESS resampling).  Returns the per-frame share of the
weight mass and of the particles on each storey."""

import math

import numpy as np

from paper_2504_18056_amd import abi

NOISE_SIGMA = (0.03, 0.03, 0.005, 0.002, 0.002, 0.008)


def run(c, policy, beta=0.05, ctx=None):
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
                     rng_frame=f, noise_sigma=NOISE_SIGMA)
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


def summary(c, mass, share, best):
    t = c["true_floor"]
    fs = c["first_seen"]
    conv = [f for f in range(fs, len(mass)) if mass[f, t] > 0.9]
    return {"first_seen_frame": int(fs),
            "floors_with_5pct_particles_before": int(np.sum(share[fs - 1] >= 0.05)),
            "mass_per_floor_before": [round(float(x), 3) for x in mass[fs - 1]],
            "true_floor_mass_end": round(float(mass[-1, t]), 4),
            "frames_to_90pct_after_first_seen": (conv[0] - fs) if conv else None,
            "representative_on_true_floor_end": bool(best[-1] == t)}
