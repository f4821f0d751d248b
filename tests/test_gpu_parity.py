"""GPU parity: the HIP filter step through the C ABI against the FP64 oracle.

Stage-wise protocol: each stage of the GPU step is checked against the oracle
started from the GPU's own inputs to that stage (likelihood and gradient at
the input poses; the pose step from the GPU's gradient; weights from the GPU's
likelihoods; resampling from those weights).  Tolerances are in parity.py.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2504_18056_amd import abi
from synth import configs

from parity import DELTA, check_eval, check_step, check_weights_resample

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = abi.mcs_create(0)
    yield c
    abi.mcs_destroy(c)


def grid_for(cfg, dtype):
    if dtype == abi.GRID_FP16:
        return oracle.quantize_fp16(cfg["grid"])
    if dtype == abi.GRID_BF16:
        return oracle.quantize_bf16(cfg["grid"])
    return cfg["grid"]


def one_step(ctx, cfg, params, dtype=abi.GRID_FP32, poses=None, logw=None, scan=None):
    poses = cfg["poses"] if poses is None else poses
    scan = cfg["scan"] if scan is None else scan
    mid = abi.mcs_init_map(ctx, abi.grid_desc(cfg["dims"], cfg["origin"], cfg["h"], dtype), cfg["grid"])
    sid = abi.mcs_session_create(ctx, mid, poses, M_max=scan.shape[0])
    try:
        if logw is not None:
            abi.mcs_set_particles(ctx, sid, logw=logw)
        abi.mcs_filter_step(ctx, sid, scan, params)
        return abi.mcs_get_particles(ctx, sid, poses.shape[0])
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)


def full_check(cfg, out, params, dtype=abi.GRID_FP32, poses=None, logw=None, scan=None,
               report=None):
    poses = cfg["poses"] if poses is None else poses
    scan = cfg["scan"] if scan is None else scan
    N = poses.shape[0]
    logw = np.full(N, -math.log(N)) if logw is None else logw
    g = grid_for(cfg, dtype)
    ref = oracle.evaluate(g, cfg["dims"], cfg["origin"], cfg["h"], params["eps"], scan, poses,
                          oob_skip=params.get("oob", 0) == abi.OOB_SKIP, delta=DELTA)
    check_eval(out["loglik"], out["grad"], ref, report=report)
    anc = out["parents"]
    check_step(poses[anc], out["grad"][anc], out["poses"], params)
    return check_weights_resample(logw, out["loglik"], params.get("beta", 1.0), params["u"], out,
                                  params.get("resample", abi.RESAMPLE_ALWAYS),
                                  params.get("ess_frac", 0.5))


@pytest.mark.parametrize("beta", [1.0, 0.002])
def test_box_room_step(ctx, box_room, beta):
    p = dict(box_room["params"], u=box_room["u"], beta=beta, resample=abi.RESAMPLE_ALWAYS)
    out = one_step(ctx, box_room, p)
    rep = {}
    res = full_check(box_room, out, p, report=rep)
    print("box_room beta=%g: %s ess=%.3f ties=%d" % (beta, rep, res["ess"], res["ties"]))
    if beta < 1:
        assert len(np.unique(out["parents"])) > 20   # a non-trivial resample


@pytest.mark.parametrize("dtype", [abi.GRID_FP16, abi.GRID_BF16])
def test_box_room_half_grids(ctx, box_room, dtype):
    p = dict(box_room["params"], u=box_room["u"], beta=0.002)
    out = one_step(ctx, box_room, p, dtype=dtype)
    rep = {}
    full_check(box_room, out, p, dtype=dtype, report=rep)
    # Quantisation error against the FP32-grid oracle is stated, not bounded.
    ref32 = oracle.evaluate(box_room["grid"], box_room["dims"], box_room["origin"], box_room["h"],
                            p["eps"], box_room["scan"], box_room["poses"])
    q = np.abs(out["loglik"] - ref32["loglik"]) / np.abs(ref32["loglik"])
    print("dtype %d: %s; vs FP32 grid: max rel l %.3g" % (dtype, rep, q.max()))


def test_ragged_sizes_and_policies(ctx):
    # N not a multiple of 64, M not a multiple of the point batching.
    c = configs.box_room(N=1000, n_rings=7, n_az=71, seed=77)
    for policy, oob in [(abi.RESAMPLE_NEVER, abi.OOB_FLOOR), (abi.RESAMPLE_ESS, abi.OOB_SKIP),
                        (abi.RESAMPLE_ALWAYS, abi.OOB_FLOOR)]:
        p = dict(c["params"], u=0.37, beta=0.01, resample=policy, oob=oob)
        full_check(c, one_step(ctx, c, p), p)


def test_post_step_likelihood(ctx):
    """post_eval: the weight uses l at the stepped pose, g stays the last gradient pass's."""
    c = configs.box_room(N=300, seed=78)
    p = dict(c["params"], u=0.5, beta=0.01, resample=abi.RESAMPLE_NEVER, post_eval=True)
    out = one_step(ctx, c, p)
    pre = oracle.evaluate(c["grid"], c["dims"], c["origin"], c["h"], p["eps"], c["scan"],
                          c["poses"], delta=DELTA)
    post = oracle.evaluate(c["grid"], c["dims"], c["origin"], c["h"], p["eps"], c["scan"],
                           out["poses"], delta=DELTA)
    check_eval(out["loglik"], out["grad"], dict(pre, loglik=post["loglik"], amb_l=post["amb_l"]))
    check_step(c["poses"], out["grad"], out["poses"], p)


@pytest.mark.parametrize("N,M", [(1, 1), (1, 300), (63, 1), (65, 513), (64, 4)])
def test_tiny_and_tail_shapes(ctx, N, M):
    c = configs.box_room(N=max(N, 2), seed=5)
    poses = c["poses"][:N]
    scan = c["scan"][:M]
    p = dict(c["params"], u=0.5, beta=0.01, resample=abi.RESAMPLE_ALWAYS)
    out = one_step(ctx, c, p, poses=poses, scan=scan)
    full_check(c, out, p, poses=poses, scan=scan)


def test_all_points_outside(ctx, box_room):
    scan = box_room["scan"] + np.float32(500.0)
    p = dict(box_room["params"], u=0.25, resample=abi.RESAMPLE_ALWAYS)
    out = one_step(ctx, box_room, p, scan=scan)
    M = scan.shape[0]
    expect = M * math.log(np.float32(p["eps"]))
    assert np.allclose(out["loglik"], expect, rtol=1e-6)
    assert np.all(out["grad"] == 0)
    # Equal weights: ESS = N and the systematic pass is the identity map.
    assert abs(out["stats"]["ess"] - box_room["poses"].shape[0]) < 1e-6
    full_check(box_room, out, p, scan=scan)


def test_deterministic_and_iteration_fusion(ctx, box_room):
    p = dict(box_room["params"], u=box_room["u"], beta=0.0, resample=abi.RESAMPLE_NEVER)
    a = one_step(ctx, box_room, p)
    b = one_step(ctx, box_room, p)
    for k in ("poses", "loglik", "grad", "logw"):
        assert np.array_equal(a[k], b[k]), k
    # Three fused passes equal three single-pass steps chained through the pose.
    p3 = dict(p, iters=3)
    f = one_step(ctx, box_room, p3)
    poses = box_room["poses"]
    for _ in range(3):
        s = one_step(ctx, box_room, p, poses=poses)
        poses = s["poses"]
    # Between launches the quaternion is renormalised once more, so the two
    # paths agree to FP32 rounding rather than bitwise.
    from parity import quat_angle
    assert np.abs(f["poses"][:, :3] - poses[:, :3]).max() < 1e-4
    assert quat_angle(f["poses"][:, 3:], poses[:, 3:]).max() < 1e-4
    assert np.allclose(f["grad"], s["grad"], rtol=1e-3, atol=1e-3 * np.abs(s["grad"]).max())


def test_prediction_matches_oracle(ctx, box_room):
    rng = np.random.default_rng(3)
    N = box_room["poses"].shape[0]
    noise = (rng.normal(size=(N, 6)) * [0.05, 0.05, 0.05, 0.017, 0.017, 0.017]).astype(np.float32)
    dq = np.array([0.999, 0.01, -0.02, 0.03])
    dq /= np.linalg.norm(dq)
    dT = np.concatenate([[0.6, -0.1, 0.02], dq]).astype(np.float32)
    p = dict(box_room["params"], u=0.5, beta=0.0, resample=abi.RESAMPLE_NEVER,
             alpha_t=0.0, alpha_r=0.0, delta_T=dT)
    mid = abi.mcs_init_map(ctx, abi.grid_desc(box_room["dims"], box_room["origin"], box_room["h"]),
                           box_room["grid"])
    sid = abi.mcs_session_create(ctx, mid, box_room["poses"], M_max=512)
    abi.mcs_filter_step(ctx, sid, box_room["scan"], p, noise=noise)
    out = abi.mcs_get_particles(ctx, sid, N)
    abi.mcs_session_destroy(ctx, sid)
    abi.mcs_release_map(ctx, mid)
    ref = oracle.predict(box_room["poses"], dT.astype(np.float64), noise)
    from parity import quat_angle, ulp32
    assert np.all(np.abs(out["poses"][:, :3] - ref[:, :3]) <= 8 * ulp32(ref[:, :3]) + 1e-6)
    assert quat_angle(out["poses"][:, 3:], ref[:, 3:]).max() < 3e-6
    # Likelihood at the predicted pose (zero gains: the step leaves the pose).
    ev = oracle.evaluate(box_room["grid"], box_room["dims"], box_room["origin"], box_room["h"],
                         p["eps"], box_room["scan"], out["poses"], delta=DELTA)
    check_eval(out["loglik"], out["grad"], ev)


def test_corridors_full_scale_sampled(ctx):
    """N = 100,000, M = 2,048 on the 512 x 512 x 128 map: sampled particles vs the oracle."""
    c = configs.corridors(N=100000, n_frames=2)
    p = dict(c["params"], iters=1, u=float(c["u"][0]), beta=1.0, resample=abi.RESAMPLE_ESS)
    out = one_step(ctx, c, p)
    rng = np.random.default_rng(0)
    # 256 random particles and the last 64 (on MI355X the last 27 tiles of 64
    # form the tail round that is spread over one wave per sub-chunk).
    idx = np.union1d(rng.choice(100000, 256, replace=False), np.arange(100000 - 64, 100000))
    ref = oracle.evaluate(c["grid"], c["dims"], c["origin"], c["h"], p["eps"], c["scan"],
                          c["poses"][idx], delta=DELTA)
    full = dict(ref)
    rep = {}
    pre_l = out["loglik"][idx]
    pre_g = out["grad"][idx]
    check_eval(pre_l, pre_g, {k: v for k, v in full.items()}, idx=np.arange(idx.size), report=rep)
    print("corridors sampled:", rep)
    anc = out["parents"]
    check_step(c["poses"][anc], out["grad"][anc], out["poses"], p)
    check_weights_resample(c["logw"], out["loglik"], 1.0, p["u"], out, abi.RESAMPLE_ESS)


def test_corridors_four_million_particles_sampled(ctx):
    """N = 2^22 + 37 (65,537 tiles, the last one ragged) on the corridors map:
    sampled particles vs the oracle, and the weights and resampling of all of
    them; the evaluation order's bounds reduce over at most 256 partial ranges
    at any N."""
    N = (1 << 22) + 37
    c = configs.corridors(N=N, n_frames=2)
    p = dict(c["params"], iters=1, u=float(c["u"][0]), beta=1.0, resample=abi.RESAMPLE_ESS)
    print("corridors N=%d M=%d" % (N, c["scan"].shape[0]), flush=True)
    out = one_step(ctx, c, p)
    rng = np.random.default_rng(1)
    idx = np.union1d(np.union1d(rng.choice(N, 256, replace=False), np.arange(N - 101, N)), np.arange(64))
    ref = oracle.evaluate(c["grid"], c["dims"], c["origin"], c["h"], p["eps"], c["scan"],
                          c["poses"][idx], delta=DELTA)
    rep = {}
    check_eval(out["loglik"][idx], out["grad"][idx], ref, idx=np.arange(idx.size), report=rep)
    print("corridors 4M sampled:", rep)
    anc = out["parents"]
    check_step(c["poses"][anc], out["grad"][anc], out["poses"], p)
    check_weights_resample(c["logw"], out["loglik"], 1.0, p["u"], out, abi.RESAMPLE_ESS)


def test_rejects_samples_outside_unit_range_and_tiny_eps(ctx, box_room):
    """Samples are likelihoods in [0, 1] and eps lies in [1e-5, 1]: the point loop
    multiplies up to four factors G + eps, which must stay normal FP32 numbers."""
    c = box_room
    desc = abi.grid_desc(c["dims"], c["origin"], c["h"])
    for bad in (1.5, -0.25, float("nan")):
        g = c["grid"].copy()
        g[3, 4, 5] = bad
        with pytest.raises(abi.McsError) as e:
            abi.mcs_init_map(ctx, desc, g)
        assert e.value.status == abi.MCS_EINVAL
    mid = abi.mcs_init_map(ctx, desc, c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=c["scan"].shape[0])
    try:
        for eps in (1e-6, 2.0):
            with pytest.raises(abi.McsError) as e:
                abi.mcs_filter_step(ctx, sid, c["scan"], dict(c["params"], eps=eps, u=0.5))
            assert e.value.status == abi.MCS_EINVAL
        # The smallest accepted eps: every factor is at least 1e-5 and the
        # product of four still normal; outside points give exactly 4 ln(eps) per four.
        p = dict(c["params"], eps=float(np.float32(1e-5)), u=0.5, beta=0.0,
                 resample=abi.RESAMPLE_NEVER)
        abi.mcs_filter_step(ctx, sid, c["scan"] + np.float32(500.0), p)
        out = abi.mcs_get_particles(ctx, sid, c["poses"].shape[0])
        expect = c["scan"].shape[0] * math.log(np.float32(1e-5))
        assert np.allclose(out["loglik"], expect, rtol=1e-6)
        assert np.all(np.isfinite(out["grad"])) and np.all(out["grad"] == 0)
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)


@pytest.mark.parametrize("N,dtype,oob", [(40000, abi.GRID_FP16, abi.OOB_FLOOR),
                                          (40000, abi.GRID_BF16, abi.OOB_SKIP),
                                          (33000, abi.GRID_FP16, abi.OOB_SKIP),
                                          (33000, abi.GRID_FP32, abi.OOB_FLOOR)])
def test_whole_rounds_and_tail_all_record_types(ctx, N, dtype, oob):
    """Sessions large enough for the main launch (N = 40,000: 625 tiles, no
    split on a 256-CU device; N = 33,000: 516 tiles, the last 4 split), every
    record type and both outside-point modes, sampled particles incl. the last."""
    c = configs.box_room(N=N, seed=91)
    p = dict(c["params"], u=0.61, beta=0.002, oob=oob, resample=abi.RESAMPLE_ESS)
    out = one_step(ctx, c, p, dtype=dtype)
    idx = np.union1d(np.arange(0, N, 211), np.arange(N - 300, N))
    g = grid_for(c, dtype)
    ref = oracle.evaluate(g, c["dims"], c["origin"], c["h"], p["eps"], c["scan"], c["poses"][idx],
                          oob_skip=oob == abi.OOB_SKIP, delta=DELTA)
    check_eval(out["loglik"][idx], out["grad"][idx], ref)
    anc = out["parents"]
    check_step(c["poses"][anc], out["grad"][anc], out["poses"], p)
    check_weights_resample(np.full(N, -math.log(N)), out["loglik"], p["beta"], p["u"], out, abi.RESAMPLE_ESS)


@pytest.mark.parametrize("dtype,oob", [(abi.GRID_FP32, abi.OOB_FLOOR), (abi.GRID_FP16, abi.OOB_FLOOR),
                                       (abi.GRID_BF16, abi.OOB_SKIP)])
def test_grid_slab_beyond_24_bits(ctx, dtype, oob):
    # (nx - 1)(ny - 1) >= 2^24 cells per slab: record offsets take full 32-bit
    # products; N = 33,000 runs whole rounds and a split tail, so both the main
    # launch and the tail kernels take that path.
    c = configs.wide_slab()
    nx, ny, _ = c["dims"]
    assert (nx - 1) * (ny - 1) >= 1 << 24
    p = dict(c["params"], u=0.61, beta=0.01, resample=abi.RESAMPLE_ALWAYS, oob=oob)
    print("wide slab dtype %d oob %d N=%d M=%d" % (dtype, oob, c["poses"].shape[0], c["scan"].shape[0]),
          flush=True)
    out = one_step(ctx, c, p, dtype=dtype)
    rep = {}
    full_check(c, out, p, dtype=dtype, report=rep)
    assert np.all(out["loglik"] > c["scan"].shape[0] * math.log(0.1))   # points inside the slab
    print("wide slab dtype %d: %s" % (dtype, rep))


def test_grid_beyond_4gib(ctx):
    # FP32 records past one buffer's 32-bit byte range (4.7 GB): record
    # addresses are formed in 64 bits.  Half the particles read records beyond
    # 4 GiB, half below; N = 33,000 runs whole rounds and a split tail.
    c = configs.beyond_4gib()
    nx, ny, nz = c["dims"]
    assert (nx + 1) * (ny + 1) * (nz + 1) * 32 > 1 << 32
    p = dict(c["params"], u=0.29, beta=0.01, resample=abi.RESAMPLE_ALWAYS)
    print("grid beyond 4 GiB N=%d M=%d" % (c["poses"].shape[0], c["scan"].shape[0]), flush=True)
    out = one_step(ctx, c, p)
    rep = {}
    full_check(c, out, p, report=rep)
    assert np.all(out["loglik"] > c["scan"].shape[0] * math.log(0.1))   # points inside the grid
    print("grid beyond 4 GiB: %s" % rep)


def test_evaluation_order_does_not_change_results(ctx):
    """Sessions of >= 4096 particles evaluate them grouped by pose cell; each
    particle's l, g and stepped pose are the same as in sessions too small to
    be reordered (bit for bit), and the grouped session still matches the oracle."""
    c = configs.box_room(N=5000, seed=93)
    p = dict(c["params"], iters=2, u=0.5, beta=0.0, resample=abi.RESAMPLE_NEVER)
    whole = one_step(ctx, c, p)
    parts = [one_step(ctx, c, p, poses=c["poses"][a:b]) for a, b in ((0, 4000), (4000, 5000))]
    for k in ("loglik", "grad", "poses"):
        assert np.array_equal(whole[k], np.concatenate([q[k] for q in parts])), k
    p1 = dict(p, iters=1, resample=abi.RESAMPLE_ALWAYS, u=0.37, beta=0.01)
    full_check(c, one_step(ctx, c, p1), p1)
