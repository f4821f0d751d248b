"""GPU parity of the keyframe-map step (Eq. 2-4 with per-particle keyframe poses).

Neighbour choice is compared bit for bit except at counted near-ties (the
kernel ranks FP32 squared distances, the oracle FP64 ones); the likelihood and gradient use the stage-wise tolerances of
parity.py, summed over the neighbours; resampling also permutes every
particle's keyframe poses.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2504_18056_amd import abi
from synth import configs

from parity import (DELTA, NB_TIE, check_loop_update, check_neighbors, check_step,
                    check_weights_resample, quat_angle)

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
    ev = dict(n_nb=p["n_neighbors"], oob_skip=p.get("oob", 0) == abi.OOB_SKIP, delta=DELTA)
    ref = oracle.kf_evaluate(grids, c["dims"], c["origins"], c["h"], p["eps"], c["scan"],
                             poses[idx], kf[idx], **ev)
    diff = check_neighbors(out["neighbors"][idx], ref, poses[idx], kf[idx])
    if diff.any():
        # Near-ties ranked the other way: compare with the oracle on the kernel's choice.
        forced = oracle.kf_evaluate(grids, c["dims"], c["origins"], c["h"], p["eps"], c["scan"],
                                    poses[idx], kf[idx], neighbors=out["neighbors"][idx], **ev)
        for k in ("loglik", "grad", "gabs", "amb_l", "amb_g"):
            ref[k][diff] = forced[k][diff]
    print("neighbour near-ties: %d of %d particles, %d ranked differently" % (
        int(np.sum(ref["nb_margin"] < NB_TIE)), idx.size, int(diff.sum())))
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
    # 128 random particles and the last 64 (on MI355X the last 14 tiles are
    # spread over one wave per sub-chunk).
    idx = np.union1d(np.random.default_rng(0).choice(50000, 128, replace=False), np.arange(50000 - 64, 50000))
    check_kf(c, out, p, idx=idx)
    check_weights_resample(c["logw"], out["loglik"], 1.0, p["u"], out, abi.RESAMPLE_ESS)


def test_ambiguous_rooms_particles_over_room_shifts(ctx):
    """Repeated identical rooms, particles spread over four copies of the initial
    cloud shifted by whole rooms: every particle against the oracle, and the
    weight held by each shift as the oracle's likelihoods give it."""
    c = configs.keyframes(N=4000, K=16, kf_points=4096, seed=33, ambiguous=True)
    room = c["scene"].rooms["room"]
    shift = np.repeat(np.arange(-2, 2), 1000)
    poses = c["poses"].copy()
    poses[:, 0] += (shift * room).astype(np.float32)
    beta = 0.01
    p = dict(c["params"], iters=1, u=0.5, beta=beta, resample=abi.RESAMPLE_NEVER)
    out = kf_step(ctx, c, p, poses=poses)
    ref = check_kf(c, out, p, poses=poses)
    check_weights_resample(c["logw"], out["loglik"], beta, p["u"], out, abi.RESAMPLE_NEVER)

    def masses(l):
        lw = beta * np.asarray(l, np.float64)
        w = np.exp(lw - lw.max())
        w /= w.sum()
        return np.array([w[shift == s].sum() for s in range(-2, 2)])

    assert np.allclose(masses(out["loglik"]), masses(ref["loglik"]), atol=1e-2)


def test_keyframe_grids_beyond_one_buffer(ctx):
    """66 FP32 keyframe grids of 128^3 exceed one buffer's 32-bit byte range, so
    the kernel reads them through 64-bit addresses (outside points read the
    map's zero record): same bounds against the oracle."""
    c = configs.keyframes(N=200, K=66, kf_points=2048, seed=38)
    stride = -(-127 ** 3 * 32 // 256) * 256
    assert stride * 66 > 0xFFFFFFE0
    p = dict(c["params"], iters=1, u=0.3, beta=0.01, resample=abi.RESAMPLE_ALWAYS)
    out = kf_step(ctx, c, p)
    check_kf(c, out, p)
    anc = out["parents"]
    check_step(c["poses"][anc], out["grad"][anc], out["poses"], p)


def test_loop_closure_out_and_back(ctx):
    """The path returns to its start: every particle sees the oldest keyframes,
    corrects its pose and propagates the step along its keyframes (Eq. 8-10)."""
    c = configs.keyframes(N=700, K=16, kf_points=4096, seed=35, out_and_back=True)
    p = dict(c["params"], iters=1, u=0.3, beta=0.01, resample=abi.RESAMPLE_NEVER,
             kf_update=abi.KF_LOOP, n_recent=4)
    out = kf_step(ctx, c, p)
    check_kf(c, out, p)
    ref = check_loop_update(c["poses"], c["kf_poses"], out, p, n_recent=4)
    assert np.all(ref["loop"] >= 0)
    moved = np.abs(out["kf_poses"][:, 1:, :3] - c["kf_poses"][:, 1:, :3]).max()
    assert moved > 1e-3


def test_loop_closure_with_tail_tiles(ctx):
    """261 tiles of 64 particles: 256 in the main launch and, on a 256-CU device,
    5 spread over one wave per sub-chunk; the loop-gated correction and its
    keyframe propagation run in both."""
    N = 261 * 64
    c = configs.keyframes(N=N, K=16, kf_points=4096, seed=39, out_and_back=True)
    p = dict(c["params"], iters=2, u=0.3, beta=0.01, resample=abi.RESAMPLE_NEVER,
             kf_update=abi.KF_LOOP, n_recent=4)
    out = kf_step(ctx, c, p)
    idx = np.union1d(np.arange(0, N, 97), np.arange(N - 5 * 64, N))
    # The first pass's likelihood and gradient at the input poses and keyframes.
    p1 = dict(p, iters=1)
    out1 = kf_step(ctx, c, p1)
    check_kf(c, out1, p1, idx=idx)
    check_loop_update(c["poses"], c["kf_poses"], out1, p1, n_recent=4)
    # Two passes: deterministic, and the same as a second run.
    again = kf_step(ctx, c, p)
    for k in ("poses", "kf_poses", "loglik", "grad", "neighbors"):
        assert np.array_equal(out[k], again[k]), k


def test_loop_gate_mixed_particles(ctx):
    """Particles whose keyframe estimate of an old keyframe sits next to them
    detect a loop; the others keep their state untouched."""
    c = configs.keyframes(N=333, K=12, kf_points=4096, seed=36)
    kf = c["kf_poses"].copy()
    poses = c["poses"]
    sel = np.arange(0, 333, 3)
    kf[sel, 2, :3] = poses[sel, :3] + np.float32(0.3)
    p = dict(c["params"], iters=1, u=0.6, beta=0.01, resample=abi.RESAMPLE_NEVER,
             kf_update=abi.KF_LOOP, n_recent=4)
    out = kf_step(ctx, c, p, kf=kf)
    check_kf(c, out, p, kf=kf)
    ref = check_loop_update(poses, kf, out, p, n_recent=4)
    loop = ref["loop"] >= 0
    assert loop[sel].all() and 0 < (~loop).sum()
    # More than W keyframes per particle to update exercises every wave's chunk.
    assert np.all(ref["loop"][sel] == 2)


def test_loop_update_is_deterministic_and_resampling_carries_it(ctx):
    c = configs.keyframes(N=500, K=16, kf_points=4096, seed=37, out_and_back=True)
    p = dict(c["params"], iters=2, u=0.45, beta=0.01, resample=abi.RESAMPLE_ALWAYS,
             kf_update=abi.KF_LOOP, n_recent=4)
    a = kf_step(ctx, c, p)
    b = kf_step(ctx, c, p)
    for k in ("poses", "kf_poses", "loglik", "grad", "parents", "logw"):
        assert np.array_equal(a[k], b[k]), k
    check_weights_resample(c["logw"], a["loglik"], 0.01, p["u"], a, abi.RESAMPLE_ALWAYS)


def test_loop_mode_rejected_without_keyframes(ctx):
    c = configs.box_room(N=64)
    mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=c["scan"].shape[0])
    try:
        with pytest.raises(abi.McsError) as e:
            abi.mcs_filter_step(ctx, sid, c["scan"], dict(c["params"], kf_update=abi.KF_LOOP))
        assert e.value.status == abi.MCS_EINVAL
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)


def test_incremental_keyframes_match_a_map_loaded_at_once(ctx):
    """Keyframes appended one at a time, each particle's keyframe pose taken from
    its pose at insertion, give the same step as the map loaded at once."""
    c = configs.keyframes(N=500, K=10, kf_points=4096, seed=38)
    K, N = 10, 500
    p = dict(c["params"], iters=2, u=0.35, beta=0.01, resample=abi.RESAMPLE_ALWAYS,
             kf_update=abi.KF_LOOP, n_recent=4)
    ref = kf_step(ctx, c, p)
    desc = [abi.grid_desc(c["dims"], c["origins"][k], c["h"]) for k in range(K)]
    mid = abi.mcs_create_keyframe_map(ctx, 16, desc[0])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=c["scan"].shape[0])
    try:
        with pytest.raises(abi.McsError) as e:           # no keyframe yet
            abi.mcs_filter_step(ctx, sid, c["scan"], p)
        assert e.value.status == abi.MCS_EINVAL
        with pytest.raises(abi.McsError) as e:           # the map has none either
            abi.mcs_session_add_keyframe(ctx, sid)
        assert e.value.status == abi.MCS_EINVAL
        for k in range(K):
            assert abi.mcs_append_keyframe(ctx, mid, desc[k], c["grids"][k]) == k
            abi.mcs_set_particles(ctx, sid, poses=np.ascontiguousarray(c["kf_poses"][:, k]))
            assert abi.mcs_session_add_keyframe(ctx, sid) == k
        abi.mcs_set_particles(ctx, sid, poses=c["poses"])
        abi.mcs_filter_step(ctx, sid, c["scan"], p)
        out = abi.mcs_get_particles(ctx, sid, N, K=K, kf_poses=True)
        out["neighbors"] = abi.mcs_get_neighbors(ctx, sid, N, p["n_neighbors"])
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)
    for key in ("poses", "kf_poses", "logw", "parents", "loglik", "grad", "neighbors"):
        assert np.array_equal(out[key], ref[key]), key


def test_keyframe_map_capacity(ctx):
    c = configs.keyframes(N=64, K=3, kf_points=2048, seed=39)
    desc = [abi.grid_desc(c["dims"], c["origins"][k], c["h"]) for k in range(3)]
    mid = abi.mcs_create_keyframe_map(ctx, 2, desc[0])
    try:
        abi.mcs_append_keyframe(ctx, mid, desc[0], c["grids"][0])
        abi.mcs_append_keyframe(ctx, mid, desc[1], c["grids"][1])
        with pytest.raises(abi.McsError) as e:
            abi.mcs_append_keyframe(ctx, mid, desc[2], c["grids"][2])
        assert e.value.status == abi.MCS_EBUSY
    finally:
        abi.mcs_release_map(ctx, mid)
