"""The measurement entry points: the gather floor (mcs_gather_floor_dev) and
the VALU issue rates (mcs_measure_issue_rates), and torch in the same process.

The gather floor runs the evaluation passes with the arithmetic cut to a
checksum of the gathered record words.  Checked here: the poses stay put
(translations bit-exact), the checksum of a particle does not depend on the
tiling of the session it sits in (whole rounds, a split tail, a small
session), repeated runs agree, and keyframe maps are refused.
"""

import math
import os

import numpy as np
import pytest
import torch

from paper_2504_18056_amd import abi
from synth import configs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DEV = torch.device("cuda:0")


def floor_run(ctx, mid, poses, scan_dev, M, p):
    sid = abi.mcs_session_create(ctx, mid, poses, M_max=M)
    try:
        abi.mcs_gather_floor_dev(ctx, sid, scan_dev, M, p)
        return abi.mcs_get_particles(ctx, sid)
    finally:
        abi.mcs_session_destroy(ctx, sid)


def test_gather_floor_keeps_poses_and_is_tiling_independent():
    c = configs.box_room(N=33000, seed=91)         # 516 tiles: the last 4 are split
    M = c["scan"].shape[0]
    scan = torch.from_numpy(np.ascontiguousarray(c["scan"])).to(DEV)
    torch.cuda.synchronize()
    p = dict(c["params"], iters=3, u=0.5)
    ctx = abi.mcs_create(0)
    try:
        mid = abi.mcs_init_map(ctx, abi.grid_desc(c["dims"], c["origin"], c["h"]), c["grid"])
        a = floor_run(ctx, mid, c["poses"], scan.data_ptr(), M, p)
        b = floor_run(ctx, mid, c["poses"], scan.data_ptr(), M, p)
        sub = np.r_[0:64, 32700:33000]
        s = floor_run(ctx, mid, c["poses"][sub], scan.data_ptr(), M, p)
        abi.mcs_release_map(ctx, mid)
        assert np.array_equal(a["poses"][:, :3], c["poses"][:, :3])
        assert np.array_equal(a["loglik"], b["loglik"])
        assert np.array_equal(s["loglik"], a["loglik"][sub])
        assert np.all(a["grad"] == 0)
        assert len(np.unique(a["loglik"])) > 100              # the checksums differ per particle
        assert np.allclose(a["logw"], -math.log(33000))       # weights untouched
        # Keyframe maps are refused.
        k = configs.keyframes(N=64, K=3, kf_points=2048, seed=39)
        descs = [abi.grid_desc(k["dims"], k["origins"][j], k["h"]) for j in range(3)]
        kmid = abi.mcs_load_keyframes(ctx, descs, [k["grids"][j] for j in range(3)])
        ksid = abi.mcs_session_create(ctx, kmid, k["poses"], M_max=M, kf_poses=k["kf_poses"])
        with pytest.raises(abi.McsError) as e:
            abi.mcs_gather_floor_dev(ctx, ksid, scan.data_ptr(), M, dict(k["params"], u=0.5))
        assert e.value.status == abi.MCS_EINVAL
        abi.mcs_session_destroy(ctx, ksid)
        abi.mcs_release_map(ctx, kmid)
    finally:
        abi.mcs_destroy(ctx)


def test_issue_rates_are_measured():
    """The per-class VALU issue rates behind the bench's issue ceilings: every
    class measured, positive and below the device's lane count x clock x 2."""
    ctx = abi.mcs_create(0)
    try:
        r = abi.mcs_measure_issue_rates(ctx)
    finally:
        abi.mcs_destroy(ctx)
    assert set(r) == set(abi.RATE_CLASSES)
    bound = 256 * 4 * 64 * 3.0e9     # far above any class on this device
    for k, v in r.items():
        assert 1e11 < v < bound, (k, v)


def test_torch_works_after_the_library_initialised_the_gpu():
    """A process that creates a context first and uses torch afterwards (the
    binding imports torch before loading the library, so both share its HIP
    runtime)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2504_18056_amd import abi\n"
            "ctx = abi.mcs_create(0)\n"
            "import torch\n"
            "x = torch.ones(8, device='cuda:0'); torch.cuda.synchronize()\n"
            "assert float(x.sum()) == 8.0\n"
            "abi.mcs_destroy(ctx)\n"
            "print('ok')\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=180)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-2000:]
