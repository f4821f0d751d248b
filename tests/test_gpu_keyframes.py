"""GPU parity of the keyframe-map step (Eq. 2-4 with per-particle keyframe poses).

Neighbour choice is compared bit for bit (both sides rank FP32 squared
distances); the likelihood and gradient use the stage-wise tolerances of
parity.py, summed over the neighbours; resampling also permutes every
particle's keyframe poses.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2504_18056_amd import abi
from synth import configs

from parity import DELTA, check_step, check_weights_resample, quat_angle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = abi.mcs_create(0)
    yield c
    abi.mcs_destroy(c)


def kf_step(ctx, c, p, dtype=abi.GRID_FP32, poses=None, kf=None):
    poses = c["poses"] if poses is None else poses
    kf = c["kf_poses"] if kf is None else kf
    K = c["grids"].shape[0]
    descs = [abi.grid_desc(c["dims"], c["origins"][k], c["h"], dtype) for k in range(K)]
    mid = abi.mcs_load_keyframes(ctx, descs, [c["grids"][k] for k in range(K)])
    N = poses.shape[0]
    sid = abi.mcs_session_create(ctx, mid, poses, M_max=c["scan"].shape[0], kf_poses=kf)
    try:
        abi.mcs_filter_step(ctx, sid, c["scan"], p)
        out = abi.mcs_get_particles(ctx, sid, N, K=K, kf_poses=True)
        out["neighbors"] = abi.mcs_get_neighbors(ctx, sid, N, p["n_neighbors"])
        return out
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)


def check_kf(c, out, p, dtype=abi.GRID_FP32, poses=None, kf=None, idx=None):
    poses = c["poses"] if poses is None else poses
    kf = c["kf_poses"] if kf is None else kf
    N = poses.shape[0]
    grids = c["grids"]
    if dtype == abi.GRID_FP16:
        grids = oracle.quantize_fp16(grids)
    elif dtype == abi.GRID_BF16:
        grids = oracle.quantize_bf16(grids)
    idx = np.arange(N) if idx is None else idx
    ref = oracle.kf_evaluate(grids, c["dims"], c["origins"], c["h"], p["eps"], c["scan"],
                             poses[idx], kf[idx], n_nb=p["n_neighbors"],
                             oob_skip=p.get("oob", 0) == abi.OOB_SKIP, delta=DELTA)
    assert np.array_equal(out["neighbors"][idx], ref["neighbors"])
    dl = np.abs(out["loglik"][idx] - ref["loglik"])
    assert np.all(dl <= 1e-5 * np.abs(ref["loglik"]) + ref["amb_l"]), dl.max()
    dg = np.abs(out["grad"][idx] - ref["grad"])
    assert np.all(dg <= 1e-4 * ref["gabs"] + ref["amb_g"] + 1e-6), (dg / ref["gabs"]).max()
    return ref


def test_keyframe_step_small(ctx):
    c = configs.keyframes(N=700, K=12, kf_points=4096, seed=31)
    p = dict(c["params"], iters=1, u=c["u"], beta=0.01, resample=abi.RESAMPLE_ALWAYS)
    out = kf_step(ctx, c, p)
    check_kf(c, out, p)
    anc = out["parents"]
    check_step(c["poses"][anc], out["grad"][anc], out["poses"], p)
    check_weights_resample(c["logw"], out["loglik"], 0.01, p["u"], out, abi.RESAMPLE_ALWAYS)
    # Keyframe poses follow their particle through resampling (bit-exact copy).
    kf = c["kf_poses"][anc].copy()
    kf[..., 3:] = np.where(kf[..., 3:4] < 0, -kf[..., 3:], kf[..., 3:])
    assert np.array_equal(out["kf_poses"][..., :3], kf[..., :3])
    assert quat_angle(out["kf_poses"][..., 3:].reshape(-1, 4), kf[..., 3:].reshape(-1, 4)).max() < 1e-6


@pytest.mark.parametrize("dtype", [abi.GRID_FP16, abi.GRID_BF16])
def test_keyframe_half_grids(ctx, dtype):
    c = configs.keyframes(N=300, K=8, kf_points=4096, seed=32, n_nb=3)
    p = dict(c["params"], iters=1, u=0.4, beta=0.01, resample=abi.RESAMPLE_NEVER, oob=abi.OOB_SKIP)
    out = kf_step(ctx, c, p, dtype=dtype)
    check_kf(c, out, p, dtype=dtype)


def test_keyframe_full_scale_sampled(ctx):
    """K = 64 keyframes of 16,384 points, N = 50,000, M = 2,048: sampled particles vs the oracle."""
    c = configs.keyframes(N=50000, K=64)
    p = dict(c["params"], iters=1, u=c["u"], beta=1.0, resample=abi.RESAMPLE_ESS)
    out = kf_step(ctx, c, p)
    idx = np.sort(np.random.default_rng(0).choice(50000, 128, replace=False))
    check_kf(c, out, p, idx=idx)
    check_weights_resample(c["logw"], out["loglik"], 1.0, p["u"], out, abi.RESAMPLE_ESS)


def test_ambiguous_rooms_keep_several_modes(ctx):
    """Repeated identical rooms: the filter keeps weight on more than one room."""
    c = configs.keyframes(N=4000, K=16, kf_points=4096, seed=33, ambiguous=True)
    p = dict(c["params"], iters=1, u=0.5, beta=0.01, resample=abi.RESAMPLE_NEVER)
    out = kf_step(ctx, c, p)
    check_kf(c, out, p, idx=np.arange(0, 4000, 40))
    assert math.isfinite(out["stats"]["ess"])
