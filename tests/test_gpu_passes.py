"""Every pass of a multi-pass step against the oracle (Sec. III-C.2, Eq. 7).

A step runs I gradient passes in one launch: pass k evaluates l and g at the
pose pass k - 1 stepped to.  The session's pass trace (mcs_session_trace)
records, per pass, the pose the pass evaluated, its l and its g; each pass is
then checked against the oracle started from that pose (teacher forcing), and
each step between passes against the oracle's step from the GPU's gradient:

* pass 0's pose against the oracle's prediction (Eq. 1) of the input state;
* pass k's l and g against oracle.evaluate at pass k's pose (tolerances of
  parity.py, face allowance DELTA);
* pass k + 1's pose against oracle.step from pass k's pose and gradient;
* the output poses against the last pass's step, gathered by the ancestors;
* weights and resampling against the oracle fed the GPU's likelihoods.

The corridors case is the benchmark's own configuration: 100,000 particles,
2,048 points, the 512 x 512 x 128 grid, odometry and prediction noise already
on the device (mcs_filter_step_dev on the session stream), 3 passes and ESS
resampling, two consecutive frames; sampled particles include the last 64
(on MI355X the tail tiles).
"""

import math

import numpy as np
import pytest

import oracle
from paper_2504_18056_amd import abi
from synth import configs

from parity import (DELTA, check_eval, check_neighbors, check_step, check_weights_resample,
                    quat_angle, ulp32)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = abi.mcs_create(0)
    yield c
    abi.mcs_destroy(c)


def assert_few_ambiguous(rep, M):
    """Points within DELTA of a cell face (where the two sides' cell choices may
    differ; the oracle's allowance covers them) must stay as rare as the FP64
    transforms' agreement makes them: a window of 2e-9 index units per axis
    holds about 6e-9 of the points.  A mismatch of the transforms themselves
    (an input or pose difference) puts thousands of points there."""
    assert rep["n_amb"] <= 2 + 1e-6 * rep["n"] * M, rep


def passes_of(p):
    return int(p["iters"]) + int(bool(p.get("post_eval", False)))


def read_state(ctx, sid):
    o = abi.mcs_get_particles(ctx, sid, poses=True, logw=True, parents=False, loglik=False,
                              grad=False, stats=False)
    return o["poses"], o["logw"]


def traces(ctx, sid, n):
    return [abi.mcs_get_pass_trace(ctx, sid, k) for k in range(n)]


def check_pass_zero(tr0, pose_in, idx, dT=None, noise=None):
    """Pass 0 evaluates the input (or predicted) pose, its quaternion normalised in FP32."""
    got = tr0["poses"][idx]
    if dT is None:
        ref = pose_in[idx].astype(np.float64)
        assert np.array_equal(got[:, :3], pose_in[idx, :3])
        assert quat_angle(got[:, 3:], ref[:, 3:]).max() < 1e-6
    else:
        ref = oracle.predict(pose_in[idx], np.asarray(dT, np.float64),
                             None if noise is None else noise[idx])
        assert np.all(np.abs(got[:, :3] - ref[:, :3]) <= 8 * ulp32(ref[:, :3]) + 1e-6)
        assert quat_angle(got[:, 3:], ref[:, 3:]).max() < 3e-6
    assert np.allclose(np.linalg.norm(got[:, 3:].astype(np.float64), axis=1), 1.0, atol=1e-6)


def check_grid_passes(c, grid, scan, p, tr, idx, reports):
    """l and g of every pass at its own pose; each step between passes."""
    n = len(tr)
    for k in range(n):
        ref = oracle.evaluate(grid, c["dims"], c["origin"], c["h"], p["eps"], scan,
                              tr[k]["poses"][idx], oob_skip=p.get("oob", 0) == abi.OOB_SKIP,
                              delta=DELTA)
        rep = {}
        check_eval(tr[k]["loglik"][idx], tr[k]["grad"][idx], ref, report=rep)
        reports.append(rep)
        if k + 1 < n:
            check_step(tr[k]["poses"][idx], tr[k]["grad"][idx], tr[k + 1]["poses"][idx], p)


def check_output(out, tr, p, idx, logw_in, beta, u, policy, ess_frac=0.5):
    """Outputs: l and g of the last passes, poses = the last step gathered by the
    ancestors, weights and resampling from the GPU's likelihoods."""
    I = int(p["iters"])
    assert np.array_equal(out["grad"], tr[I - 1]["grad"])
    assert np.array_equal(out["loglik"], tr[-1]["loglik"])
    anc = out["parents"]
    sel = np.flatnonzero(np.isin(anc, idx))
    if p.get("post_eval", False):
        # The post-step pass holds the stepped pose; the output is its copy.
        want = tr[I]["poses"][anc[sel]].copy()
        want[:, 3:] = np.where(want[:, 3:4] < 0, -want[:, 3:], want[:, 3:])
        assert np.array_equal(out["poses"][sel], want)
    else:
        check_step(tr[I - 1]["poses"][anc[sel]], tr[I - 1]["grad"][anc[sel]], out["poses"][sel], p)
    return check_weights_resample(logw_in, out["loglik"], beta, u, out, policy, ess_frac)


def grid_for(c, dtype):
    if dtype == abi.GRID_FP16:
        return oracle.quantize_fp16(c["grid"])
    if dtype == abi.GRID_BF16:
        return oracle.quantize_bf16(c["grid"])
    return c["grid"]


@pytest.mark.parametrize("case", ["box3", "ragged_post_skip_fp16", "predict_bf16"])
def test_every_pass_of_a_fused_step(ctx, case):
    if case == "box3":
        c = configs.box_room(N=1024)
        p = dict(c["params"], iters=3, u=c["u"], beta=0.002, resample=abi.RESAMPLE_ALWAYS)
        dtype, scan, noise, dT = abi.GRID_FP32, c["scan"], None, None
    elif case == "ragged_post_skip_fp16":
        c = configs.box_room(N=1000, n_rings=7, n_az=71, seed=79)
        p = dict(c["params"], iters=2, u=0.41, beta=0.01, resample=abi.RESAMPLE_ESS,
                 post_eval=True, oob=abi.OOB_SKIP)
        dtype, scan, noise, dT = abi.GRID_FP16, c["scan"], None, None
    else:
        c = configs.box_room(N=777, seed=80)
        rng = np.random.default_rng(80)
        N = c["poses"].shape[0]
        noise = (rng.normal(size=(N, 6)) * [0.05, 0.05, 0.05, 0.017, 0.017, 0.017]).astype(np.float32)
        dq = np.array([0.999, 0.01, -0.02, 0.03])
        dT = np.concatenate([[0.4, -0.1, 0.02], dq / np.linalg.norm(dq)]).astype(np.float32)
        p = dict(c["params"], iters=4, u=0.77, beta=0.005, resample=abi.RESAMPLE_ALWAYS, delta_T=dT)
        dtype, scan = abi.GRID_BF16, c["scan"]
    N = c["poses"].shape[0]
    mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"], dtype), c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=scan.shape[0])
    try:
        abi.mcs_session_trace(ctx, sid, passes_of(p))
        abi.mcs_filter_step(ctx, sid, scan, p, noise=noise)
        out = abi.mcs_get_particles(ctx, sid)
        tr = traces(ctx, sid, passes_of(p))
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)
    idx = np.arange(N)
    check_pass_zero(tr[0], c["poses"], idx, dT=dT, noise=noise)
    reports = []
    check_grid_passes(c, grid_for(c, dtype), scan, p, tr, idx, reports)
    res = check_output(out, tr, p, idx, np.full(N, -math.log(N)), p["beta"], p["u"], p["resample"])
    print("%s: per pass %s; ess %.2f ties %d" % (case, reports, res["ess"], res["ties"]))
    for r in reports:
        assert_few_ambiguous(r, M=scan.shape[0])


def test_corridors_benchmark_configuration_every_pass(ctx):
    """The benchmark's step (N = 100,000, M = 2,048, 3 passes, prediction with
    device-resident odometry noise, ESS resampling) for two consecutive frames,
    every pass of each checked on sampled particles."""
    import torch
    dev = torch.device("cuda:0")
    c = configs.corridors(N=100000, n_frames=3)
    N, M = c["poses"].shape[0], c["scans"].shape[1]
    scans = torch.from_numpy(np.ascontiguousarray(c["scans"])).to(dev)
    noise_h = [configs.prediction_noise(N, f, c["noise_sigma"], c["noise_seed"]) for f in (1, 2)]
    noise = [torch.from_numpy(x).to(dev) for x in noise_h]
    torch.cuda.synchronize()
    base = dict(c["params"], resample=abi.RESAMPLE_ESS, ess_frac=0.5)
    rng = np.random.default_rng(0)
    idx = np.union1d(rng.choice(N, 256, replace=False), np.arange(N - 64, N))
    mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M)
    try:
        stream = abi.mcs_session_stream(ctx, sid)
        abi.mcs_session_trace(ctx, sid, passes_of(base))
        for k, f in enumerate((1, 2)):
            pose_in, logw_in = read_state(ctx, sid)
            p = dict(base, u=float(c["u"][f]), delta_T=c["odometry"][f])
            print("corridors frame %d: N=%d M=%d passes=%d" % (f, N, M, passes_of(p)), flush=True)
            abi.mcs_filter_step_dev(ctx, sid, scans[f].data_ptr(), M, p,
                                    noise_dev_ptr=noise[k].data_ptr(), stream=stream)
            out = abi.mcs_get_particles(ctx, sid)
            tr = traces(ctx, sid, passes_of(p))
            check_pass_zero(tr[0], pose_in, idx, dT=c["odometry"][f], noise=noise_h[k])
            reports = []
            check_grid_passes(c, c["grid"], c["scans"][f], p, tr, idx, reports)
            res = check_output(out, tr, p, idx, logw_in, 1.0, p["u"], abi.RESAMPLE_ESS)
            print("corridors frame %d: per pass %s; ess %.1f resampled %s ties %d" % (
                f, reports, res["ess"], out["stats"]["resampled"], res["ties"]), flush=True)
            for r in reports:
                assert_few_ambiguous(r, M=M)
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)


def test_keyframe_map_every_pass(ctx):
    """Keyframe map (K = 12, 4 neighbours chosen once per frame at pass 0's
    pose), 3 passes: each pass against the oracle on the kernel's neighbours."""
    c = configs.keyframes(N=700, K=12, kf_points=4096, seed=31)
    p = dict(c["params"], iters=3, u=c["u"], beta=0.01, resample=abi.RESAMPLE_ALWAYS)
    K = c["grids"].shape[0]
    N = c["poses"].shape[0]
    descs = [abi.grid_desc(c["dims"], c["origins"][k], c["h"]) for k in range(K)]
    mid = abi.mcs_load_keyframes(ctx, descs, [c["grids"][k] for k in range(K)])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=c["scan"].shape[0], kf_poses=c["kf_poses"])
    try:
        abi.mcs_session_trace(ctx, sid, 3)
        abi.mcs_filter_step(ctx, sid, c["scan"], p)
        out = abi.mcs_get_particles(ctx, sid)
        nb = abi.mcs_get_neighbors(ctx, sid)
        tr = traces(ctx, sid, 3)
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)
    idx = np.arange(N)
    check_pass_zero(tr[0], c["poses"], idx)
    sel = oracle.kf_evaluate(c["grids"], c["dims"], c["origins"], c["h"], p["eps"], c["scan"][:1],
                             tr[0]["poses"], c["kf_poses"], n_nb=p["n_neighbors"])
    check_neighbors(nb, sel, tr[0]["poses"], c["kf_poses"])
    for k in range(3):
        ref = oracle.kf_evaluate(c["grids"], c["dims"], c["origins"], c["h"], p["eps"], c["scan"],
                                 tr[k]["poses"], c["kf_poses"], n_nb=p["n_neighbors"], delta=DELTA,
                                 neighbors=nb)
        rep = {}
        check_eval(tr[k]["loglik"], tr[k]["grad"], ref, report=rep)
        print("keyframes pass %d: %s" % (k, rep))
        assert_few_ambiguous(rep, M=c["scan"].shape[0] * p["n_neighbors"])
        if k < 2:
            check_step(tr[k]["poses"], tr[k]["grad"], tr[k + 1]["poses"], p)
    check_output(out, tr, p, idx, c["logw"], 0.01, p["u"], abi.RESAMPLE_ALWAYS)


def test_trace_errors(ctx, box_room):
    c = box_room
    mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
    sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=c["scan"].shape[0])
    try:
        with pytest.raises(abi.McsError):                 # no trace yet
            abi.mcs_get_pass_trace(ctx, sid, 0)
        abi.mcs_session_trace(ctx, sid, 2)
        with pytest.raises(abi.McsError) as e:            # more passes than the trace holds
            abi.mcs_filter_step(ctx, sid, c["scan"], dict(c["params"], iters=3, u=0.5))
        assert e.value.status == abi.MCS_EINVAL
        with pytest.raises(abi.McsError):
            abi.mcs_get_pass_trace(ctx, sid, 2)
        abi.mcs_session_trace(ctx, sid, 0)
        abi.mcs_filter_step(ctx, sid, c["scan"], dict(c["params"], iters=3, u=0.5))
        with pytest.raises(abi.McsError):
            abi.mcs_get_pass_trace(ctx, sid, 0)
    finally:
        abi.mcs_session_destroy(ctx, sid)
        abi.mcs_release_map(ctx, mid)
