"""The allocation-free step (mcs_filter_step_noalloc) against the session step.

Both run the same kernels in the same order on the same inputs, so every
output must be bit-identical: the step from caller-held state with the
temporaries in the library's static area, and mcs_filter_step_dev on a
session.  Two calls in a row, the second with fewer particles and points
(the static area keeps the first call's contents), both with prediction
noise and resampling; the second call's particle count also takes the split
small-session path, whose partial sums live in the static area too.
"""

import math

import numpy as np
import pytest
import torch

from paper_2504_18056_amd import abi
from synth import configs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def session_step(ctx, mid, poses, scan, noise, p):
    sid = abi.mcs_session_create(ctx, mid, poses, M_max=scan.shape[0])
    try:
        s = torch.from_numpy(np.ascontiguousarray(scan)).to(DEV)
        n = torch.from_numpy(np.ascontiguousarray(noise)).to(DEV)
        torch.cuda.synchronize()
        abi.mcs_filter_step_dev(ctx, sid, s.data_ptr(), scan.shape[0], p, noise_dev_ptr=n.data_ptr())
        out = abi.mcs_get_particles(ctx, sid)
    finally:
        abi.mcs_session_destroy(ctx, sid)
    return out


def noalloc_step(ctx, mid, poses, scan, noise, p):
    N, M = poses.shape[0], scan.shape[0]
    pose = torch.from_numpy(np.ascontiguousarray(poses.T)).to(DEV)          # [7][N]
    logw = torch.full((N,), -math.log(N), dtype=torch.float64, device=DEV)
    loglik = torch.full((N,), float("nan"), dtype=torch.float32, device=DEV)
    grad = torch.full((6, N), float("nan"), dtype=torch.float32, device=DEV)
    parents = torch.full((N,), -7, dtype=torch.int32, device=DEV)
    stats = torch.zeros(8, dtype=torch.float64, device=DEV)                 # one mcs_step_stats (64 B)
    s = torch.from_numpy(np.ascontiguousarray(scan)).to(DEV)
    n = torch.from_numpy(np.ascontiguousarray(noise)).to(DEV)
    torch.cuda.synchronize()
    abi.mcs_filter_step_noalloc(ctx, mid, N, pose.data_ptr(), logw.data_ptr(), loglik.data_ptr(),
                                grad.data_ptr(), parents.data_ptr(), s.data_ptr(), M, p,
                                noise_dev=n.data_ptr(), stats_dev=stats.data_ptr())
    torch.cuda.synchronize()
    P = pose.cpu().numpy().T.copy()
    P[:, 3:] = np.where(P[:, 3:4] < 0, -P[:, 3:], P[:, 3:])                 # as mcs_get_particles
    st = abi.StepStats.from_buffer_copy(stats.cpu().numpy().tobytes())
    return dict(poses=P, logw=logw.cpu().numpy(), loglik=loglik.cpu().numpy(),
                grad=grad.cpu().numpy().T.copy(), parents=parents.cpu().numpy(),
                stats=dict(lse=st.lse, ess=st.ess, resampled=bool(st.resampled), best=st.best,
                           best_pose=np.array(st.best_pose[:], np.float32)))


def test_noalloc_step_matches_the_session_step_twice():
    big = configs.box_room(N=40000, seed=95)
    small = configs.box_room(N=20000, n_rings=6, n_az=50, seed=96)   # 313 tiles: split whole
    ctx = abi.mcs_create(0)
    try:
        for c, beta in ((big, 0.002), (small, 0.01)):
            N, M = c["poses"].shape[0], c["scan"].shape[0]
            print("noalloc: N=%d M=%d" % (N, M), flush=True)
            rng = np.random.default_rng(N)
            noise = (rng.normal(size=(N, 6)) * [0.05, 0.05, 0.05, 0.017, 0.017, 0.017]).astype(np.float32)
            dq = np.array([0.999, 0.01, -0.02, 0.03])
            dT = np.concatenate([[0.3, -0.1, 0.02], dq / np.linalg.norm(dq)]).astype(np.float32)
            p = dict(c["params"], iters=3, u=0.43, beta=beta, resample=abi.RESAMPLE_ALWAYS,
                     delta_T=dT)
            mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
            try:
                ref = session_step(ctx, mid, c["poses"], c["scan"], noise, p)
                got = noalloc_step(ctx, mid, c["poses"], c["scan"], noise, p)
            finally:
                abi.mcs_release_map(ctx, mid)
            for k in ("poses", "logw", "loglik", "grad", "parents"):
                assert np.array_equal(got[k], ref[k]), k
            for k in ("lse", "ess", "resampled", "best"):
                assert got["stats"][k] == ref["stats"][k], k
            assert np.array_equal(got["stats"]["best_pose"], ref["stats"]["best_pose"])
            assert len(np.unique(got["parents"])) > 10
    finally:
        abi.mcs_destroy(ctx)


def test_noalloc_step_rejects_sizes_beyond_the_static_area():
    c = configs.box_room(N=64, seed=97)
    ctx = abi.mcs_create(0)
    try:
        mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
        p = dict(c["params"], u=0.5)
        x = torch.zeros(16, dtype=torch.float64, device=DEV)
        ptr = x.data_ptr()
        for N, M in ((abi.NOALLOC_MAX_PARTICLES + 1, 512), (64, abi.NOALLOC_MAX_POINTS + 1), (0, 512)):
            with pytest.raises(abi.McsError) as e:
                abi.mcs_filter_step_noalloc(ctx, mid, N, ptr, ptr, ptr, ptr, ptr, ptr, M, p)
            assert e.value.status == abi.MCS_EINVAL
            assert "static area" in str(e.value) or N == 0
        abi.mcs_release_map(ctx, mid)
    finally:
        abi.mcs_destroy(ctx)
