"""GPU tests of the serving loop: continuous batching of many sessions.

Each session's result in the batched mix must equal, bit for bit, the result
of running the same frames alone through mcs_filter_step_dev: the batched
persistent kernels run the same per-session device code with the same block
decomposition and fixed reduction order.  Each tick replays a captured HIP
graph, so these tests replay it many times, with eager work and
synchronisation in between, and check every replay.
"""

import math

import numpy as np
import pytest
import torch

from paper_2504_18056_amd import abi
from synth import configs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = abi.mcs_create(0)
    yield c
    abi.mcs_destroy(c)


def make_sessions(ctx, specs, dtype=abi.GRID_FP16, frames=3):
    """specs: list of (N, rings, grid_n, seed).  Returns per-session dicts."""
    out = []
    for N, rings, grid_n, seed in specs:
        c = configs.box_room(N=N, seed=seed, grid_n=grid_n, n_rings=rings)
        rng = np.random.default_rng(seed)
        M = c["scan"].shape[0]
        scans = np.stack([c["scan"]] + [c["scan"] + rng.normal(0, 0.01, c["scan"].shape).astype(np.float32)
                                         for _ in range(frames - 1)])
        noise = (rng.normal(size=(frames, N, 6)) * [0.02, 0.02, 0.02, 0.005, 0.005, 0.005]).astype(np.float32)
        mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"], dtype), c["grid"])
        sid = abi.mcs_session_create(ctx, mid, c["poses"], M_max=M)
        dq = np.array([0.9999, 0.0, 0.0, 0.0141], np.float32)
        params = [dict(c["params"], iters=2, u=float(0.1 + 0.2 * f), beta=0.01, resample=abi.RESAMPLE_ESS,
                       ess_frac=0.5, delta_T=np.array([0.05, 0.0, 0.0, *dq], np.float32))
                  for f in range(frames)]
        if seed in PRUNING_SEEDS:
            # Dead-particle pruning with noise drawn on the device.
            for f, q in enumerate(params):
                q.update(resample=abi.RESAMPLE_PRUNE, beta=0.2, noise_mode=abi.NOISE_DEVICE,
                         rng_seed=seed, rng_frame=f, noise_sigma=(0.02, 0.02, 0.02, 0.005, 0.005, 0.005))
        out.append(dict(cfg=c, N=N, M=M, mid=mid, sid=sid, params=params,
                        scans=torch.from_numpy(scans).to(DEV), noise=torch.from_numpy(noise).to(DEV)))
    torch.cuda.synchronize()
    return out


def snapshot(ctx, s):
    o = abi.mcs_get_particles(ctx, s["sid"], s["N"])
    return {k: o[k].copy() for k in ("poses", "logw", "parents", "loglik", "grad")} | {
        "lse": o["stats"]["lse"], "ess": o["stats"]["ess"], "pruned": o["stats"]["pruned"]}


def reset(ctx, s):
    abi.mcs_set_particles(ctx, s["sid"], poses=s["cfg"]["poses"], logw=np.full(s["N"], -math.log(s["N"])))


def run_alone(ctx, sessions, frames):
    ref = []
    for s in sessions:
        reset(ctx, s)
        snaps = []
        for f in range(frames):
            abi.mcs_filter_step_dev(ctx, s["sid"], s["scans"][f].data_ptr(), s["M"], s["params"][f],
                                    noise_dev_ptr=s["noise"][f].data_ptr())
            snaps.append(snapshot(ctx, s))
        ref.append(snaps)
    return ref


def assert_same(a, b, what):
    for k in ("poses", "logw", "parents", "loglik", "grad"):
        assert np.array_equal(a[k], b[k]), "%s: %s differs" % (what, k)
    assert a["lse"] == b["lse"] and a["ess"] == b["ess"] and a["pruned"] == b["pruned"], what


PRUNING_SEEDS = (204, 206)
SPECS = [(1000, 8, 64, 201), (3000, 16, 96, 202), (64, 8, 64, 203), (12345, 32, 128, 204),
         (257, 12, 64, 205), (40000, 20, 128, 206)]


@pytest.mark.parametrize("mode", [abi.SERVE_BATCHED, abi.SERVE_CONCURRENT, abi.SERVE_SERIAL])
def test_each_session_same_alone_and_in_the_mix(ctx, mode):
    frames = 3
    sessions = make_sessions(ctx, SPECS, frames=frames)
    try:
        ref = run_alone(ctx, sessions, frames)
        for s in sessions:
            reset(ctx, s)
        srv = abi.mcs_server_create(ctx, mode=mode, dtype=abi.GRID_FP16, max_batch=8)
        try:
            # Frame by frame: one tick (graph replay) per frame, checked each time.
            for f in range(frames):
                for s in sessions:
                    abi.mcs_server_submit(srv, s["sid"], s["scans"][f].data_ptr(), s["M"], s["params"][f],
                                          noise_dev_ptr=s["noise"][f].data_ptr())
                abi.mcs_server_drain(srv)
                for k, s in enumerate(sessions):
                    assert_same(ref[k][f], snapshot(ctx, s), "session %d frame %d" % (k, f))
            # All frames at once: sessions spread over consecutive ticks in varying mixes.
            for s in sessions:
                reset(ctx, s)
            order = [(k, f) for f in range(frames) for k in range(len(sessions))]
            rng = np.random.default_rng(5)
            rng.shuffle(order)
            # Keep each session's frames in order.
            nxt = [0] * len(sessions)
            for k, _ in order:
                f = nxt[k]
                nxt[k] += 1
                s = sessions[k]
                abi.mcs_server_submit(srv, s["sid"], s["scans"][f].data_ptr(), s["M"], s["params"][f],
                                      noise_dev_ptr=s["noise"][f].data_ptr())
            abi.mcs_server_drain(srv)
            for k, s in enumerate(sessions):
                assert_same(ref[k][frames - 1], snapshot(ctx, s), "session %d (mixed)" % k)
            assert any(ref[k][f]["pruned"] > 0 for k in range(len(sessions)) for f in range(frames))
            st = abi.mcs_server_stats_get(srv)
            assert st["requests"] == 2 * frames * len(sessions)
            if mode != abi.SERVE_SERIAL:
                assert st["max_batch_seen"] > 1
        finally:
            abi.mcs_server_destroy(srv)
    finally:
        for s in sessions:
            abi.mcs_session_destroy(ctx, s["sid"])
            abi.mcs_release_map(ctx, s["mid"])


def test_request_times_are_ordered(ctx):
    sessions = make_sessions(ctx, SPECS[:3], frames=2)
    try:
        srv = abi.mcs_server_create(ctx, dtype=abi.GRID_FP16)
        try:
            ids = []
            for f in range(2):
                for s in sessions:
                    ids.append(abi.mcs_server_submit(srv, s["sid"], s["scans"][f].data_ptr(), s["M"],
                                                     s["params"][f], noise_dev_ptr=s["noise"][f].data_ptr()))
            abi.mcs_server_drain(srv)
            for rid in ids:
                t = abi.mcs_server_times(srv, rid)
                assert 0 < t["submit_ns"] <= t["launch_ns"] <= t["done_ns"]
        finally:
            abi.mcs_server_destroy(srv)
    finally:
        for s in sessions:
            abi.mcs_session_destroy(ctx, s["sid"])
            abi.mcs_release_map(ctx, s["mid"])


def test_admission_by_hbm_budget():
    c = configs.box_room(N=2000, grid_n=64)
    probe = abi.mcs_create(0)
    mid = abi.mcs_init_map(probe, abi.grid_desc(c["dims"], c["origin"], c["h"], abi.GRID_FP16), c["grid"])
    map_bytes = abi.mcs_memory_in_use(probe)
    sess_bytes = abi.mcs_session_bytes(probe, mid, 2000, 512)
    abi.mcs_destroy(probe)
    # Room for the map and exactly two sessions.
    ctx = abi.mcs_create(0, hbm_budget_bytes=map_bytes + 2 * sess_bytes + sess_bytes // 2)
    try:
        mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"], abi.GRID_FP16), c["grid"])
        a = abi.mcs_session_create(ctx, mid, c["poses"], M_max=512)
        b = abi.mcs_session_create(ctx, mid, c["poses"], M_max=512)
        with pytest.raises(abi.McsError) as e:
            abi.mcs_session_create(ctx, mid, c["poses"], M_max=512)
        assert e.value.status == abi.MCS_EBUDGET
        with pytest.raises(abi.McsError) as e:
            abi.mcs_release_map(ctx, mid)
        assert e.value.status == abi.MCS_EBUSY
        abi.mcs_session_destroy(ctx, a)
        d = abi.mcs_session_create(ctx, mid, c["poses"], M_max=512)   # admitted once memory frees
        abi.mcs_session_destroy(ctx, b)
        abi.mcs_session_destroy(ctx, d)
        assert abi.mcs_memory_in_use(ctx) == map_bytes
    finally:
        abi.mcs_destroy(ctx)


def test_server_rejects_other_dtype(ctx):
    s = make_sessions(ctx, SPECS[:1], dtype=abi.GRID_FP32, frames=1)[0]
    try:
        srv = abi.mcs_server_create(ctx, dtype=abi.GRID_FP16)
        try:
            with pytest.raises(abi.McsError) as e:
                abi.mcs_server_submit(srv, s["sid"], s["scans"][0].data_ptr(), s["M"], s["params"][0])
            assert e.value.status == abi.MCS_EINVAL
        finally:
            abi.mcs_server_destroy(srv)
    finally:
        abi.mcs_session_destroy(ctx, s["sid"])
        abi.mcs_release_map(ctx, s["mid"])


@pytest.mark.parametrize("dtype,oob", [(abi.GRID_FP16, abi.OOB_SKIP), (abi.GRID_FP32, abi.OOB_FLOOR),
                                       (abi.GRID_BF16, abi.OOB_FLOOR)])
def test_batched_record_types_and_skip_same_alone(ctx, dtype, oob):
    # Servers of the other record types, and one whose sessions skip outside
    # points: the batched kernels' variants against each session stepped alone.
    frames = 2
    sessions = make_sessions(ctx, [(1000, 8, 64, 211), (257, 12, 64, 212), (3000, 16, 96, 213)],
                             dtype=dtype, frames=frames)
    for s in sessions:
        for q in s["params"]:
            q["oob"] = oob
    try:
        ref = run_alone(ctx, sessions, frames)
        for s in sessions:
            reset(ctx, s)
        srv = abi.mcs_server_create(ctx, mode=abi.SERVE_BATCHED, dtype=dtype, oob=oob, max_batch=8)
        try:
            for f in range(frames):
                for s in sessions:
                    abi.mcs_server_submit(srv, s["sid"], s["scans"][f].data_ptr(), s["M"], s["params"][f],
                                          noise_dev_ptr=s["noise"][f].data_ptr())
                abi.mcs_server_drain(srv)
                for k, s in enumerate(sessions):
                    assert_same(ref[k][f], snapshot(ctx, s), "dtype %d oob %d session %d frame %d" % (dtype, oob, k, f))
            assert abi.mcs_server_stats_get(srv)["max_batch_seen"] > 1
        finally:
            abi.mcs_server_destroy(srv)
    finally:
        for s in sessions:
            abi.mcs_session_destroy(ctx, s["sid"])
            abi.mcs_release_map(ctx, s["mid"])


def test_wide_grid_session_in_the_batched_server(ctx):
    # A grid whose slabs hold 2^24 records or more needs the BIG kernels, which
    # the batched tick kernels do not take: such a session runs in the
    # large-session lane, with the same results as stepped alone, beside a
    # session that runs in the ticks.
    frames = 2
    w = configs.wide_slab(N=1000, M=300)
    rng = np.random.default_rng(5)
    mid = abi.mcs_init_map(ctx, abi.grid_desc(w["dims"], w["origin"], w["h"], abi.GRID_FP16), w["grid"])
    sid = abi.mcs_session_create(ctx, mid, w["poses"], M_max=300)
    scans = torch.from_numpy(np.stack([w["scan"], w["scan"] + rng.normal(0, 0.01, w["scan"].shape).astype(np.float32)])).to(DEV)
    noise = torch.from_numpy((rng.normal(size=(frames, 1000, 6)) * 0.005).astype(np.float32)).to(DEV)
    wide = dict(cfg=w, N=1000, M=300, mid=mid, sid=sid, scans=scans, noise=noise,
                params=[dict(w["params"], iters=2, u=0.3 + 0.2 * f, beta=0.01, resample=abi.RESAMPLE_ALWAYS)
                        for f in range(frames)])
    torch.cuda.synchronize()
    sessions = [wide] + make_sessions(ctx, [(1000, 8, 64, 221)], dtype=abi.GRID_FP16, frames=frames)
    try:
        ref = run_alone(ctx, sessions, frames)
        for s in sessions:
            reset(ctx, s)
        srv = abi.mcs_server_create(ctx, mode=abi.SERVE_BATCHED, dtype=abi.GRID_FP16, max_batch=8)
        try:
            for f in range(frames):
                for s in sessions:
                    abi.mcs_server_submit(srv, s["sid"], s["scans"][f].data_ptr(), s["M"], s["params"][f],
                                          noise_dev_ptr=s["noise"][f].data_ptr())
                abi.mcs_server_drain(srv)
                for k, s in enumerate(sessions):
                    assert_same(ref[k][f], snapshot(ctx, s), "session %d frame %d" % (k, f))
        finally:
            abi.mcs_server_destroy(srv)
    finally:
        for s in sessions:
            abi.mcs_session_destroy(ctx, s["sid"])
            abi.mcs_release_map(ctx, s["mid"])
