"""Pins for the oracle's loop-gated keyframe update (Sec. III-C.2, Eq. 8-10).

References independent of the oracle: the discount ratios are written out by
hand for a straight, evenly spaced trajectory, path lengths come from numpy's
cumulative sums of segment lengths, and every updated pose is the 4x4 product
T_k expm(twist(ratio * psi)) with scipy's matrix exponential.
"""

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle

from test_oracle_se3 import twist

# Step constants large enough that psi = alpha * g stays inside the clamps.
PARAMS = dict(alpha_t=1.0, alpha_r=1.0, rho_max=10.0, phi_max=1.0)


def pose_mat(p):
    T = np.eye(4)
    q = np.asarray(p[3:], np.float64)
    q = q / np.linalg.norm(q)
    T[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    T[:3, 3] = p[:3]
    return T


def mat_pose(T):
    x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
    q = np.array([w, x, y, z])
    return np.concatenate([T[:3, 3], q if w >= 0 else -q])


def same_pose(a, b, tol=1e-12):
    qa, qb = a[3:] * np.sign(a[3] or 1.0), b[3:] * np.sign(b[3] or 1.0)
    return np.allclose(a[:3], b[:3], rtol=0, atol=tol) and np.allclose(qa, qb, rtol=0, atol=tol)


def ident(t):
    return np.array([*t, 1.0, 0.0, 0.0, 0.0], np.float32)


def test_straight_path_ratios_by_hand():
    K, s, d = 10, 2.0, 0.5
    kf = np.stack([ident((k * s, 0.0, 0.0)) for k in range(K)])[None]
    pose = ident(((K - 1) * s + d, 0.0, 0.0))[None]
    g = np.array([[0.3, -0.2, 0.1, 0.0, 0.0, 0.0]])
    nb = np.array([[2, K - 1, K - 2]], np.int32)           # keyframe 2 is old: a loop
    r = oracle.kf_loop_update(pose, kf, g, nb, PARAMS, n_recent=3)
    assert r["loop"][0] == 2
    assert np.allclose(r["poses"][0, :3], pose[0, :3] + g[0, :3], atol=1e-12)
    for k in range(K):
        ratio = 0.0 if k <= 2 else (k - 2) * s / ((K - 3) * s + d)
        assert np.allclose(r["kf_poses"][0, k, :3], kf[0, k, :3] + ratio * g[0, :3], atol=1e-12)
        assert np.allclose(r["kf_poses"][0, k, 3:], [1, 0, 0, 0], atol=1e-15)
    # The oldest neighbour and everything before it stay exactly where they were.
    assert np.array_equal(r["kf_poses"][0, :3], kf[0, :3].astype(np.float64))


def random_pose(rng, spread=10.0):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return np.array([*(rng.normal(size=3) * spread), *q], np.float32)


def test_general_update_against_matrix_exponential():
    rng = np.random.default_rng(11)
    N, K, n_nb = 40, 16, 4
    poses = np.stack([random_pose(rng) for _ in range(N)])
    kf = np.stack([np.stack([random_pose(rng) for _ in range(K)]) for _ in range(N)])
    g = rng.normal(size=(N, 6)) * [0.5, 0.5, 0.5, 0.2, 0.2, 0.2]
    nb = np.stack([rng.choice(K, n_nb, replace=False) for _ in range(N)]).astype(np.int32)
    nb[::5] = rng.permutation(np.arange(K - n_nb, K))      # only recent neighbours: no loop
    r = oracle.kf_loop_update(poses, kf, g, nb, PARAMS, n_recent=n_nb)
    n_loop = 0
    for i in range(N):
        o = nb[i].min()
        if o >= K - n_nb:
            assert r["loop"][i] == -1
            assert same_pose(r["poses"][i], poses[i].astype(np.float64), 1e-7)
            continue
        n_loop += 1
        assert r["loop"][i] == o
        psi = r["psi"][i]
        assert np.allclose(psi, g[i], atol=1e-15)            # inside the clamps: psi = g
        assert same_pose(r["poses"][i], mat_pose(pose_mat(poses[i]) @ expm(twist(psi))))
        seg = np.linalg.norm(np.diff(kf[i, o:, :3].astype(np.float64), axis=0), axis=1)
        dk = np.concatenate([[0.0], np.cumsum(seg)])
        dt = dk[-1] + np.linalg.norm(poses[i, :3].astype(np.float64) - kf[i, K - 1, :3])
        for k in range(K):
            want = pose_mat(kf[i, k])
            if k > o:
                want = want @ expm(twist(dk[k - o] / dt * psi))
            assert same_pose(r["kf_poses"][i, k], mat_pose(want), 1e-10), (i, k)
    assert 0 < n_loop < N


def test_rotation_only_step_along_a_bent_path():
    rng = np.random.default_rng(12)
    K = 8
    pts = np.cumsum(rng.normal(size=(K + 1, 3)), axis=0)
    kf = np.stack([ident(p) for p in pts[:K]])[None]
    pose = ident(pts[K])[None]
    phi = np.array([0.05, -0.02, 0.03])
    g = np.concatenate([[0.0, 0.0, 0.0], phi])[None]
    r = oracle.kf_loop_update(pose, kf, g, np.array([[0, 6, 7]], np.int32), PARAMS, n_recent=3)
    seg = np.linalg.norm(np.diff(pts.astype(np.float32).astype(np.float64), axis=0), axis=1)
    ratio = np.concatenate([[0.0], np.cumsum(seg[:K - 1])]) / seg.sum()
    for k in range(K):
        x, y, z, w = Rotation.from_rotvec(ratio[k] * phi).as_quat()
        assert np.allclose(r["kf_poses"][0, k, 3:], [w, x, y, z], atol=1e-14)
        assert np.allclose(r["kf_poses"][0, k, :3], kf[0, k, :3], atol=1e-14)


def test_recent_neighbours_only_change_nothing():
    rng = np.random.default_rng(13)
    K = 12
    kf = np.stack([np.stack([random_pose(rng) for _ in range(K)]) for _ in range(3)])
    poses = np.stack([random_pose(rng) for _ in range(3)])
    g = rng.normal(size=(3, 6))
    nb = np.array([[K - 1, K - 2, K - 3], [K - 3, K - 1, K - 2], [K - 2, K - 3, K - 1]], np.int32)
    r = oracle.kf_loop_update(poses, kf, g, nb, PARAMS, n_recent=3)
    assert np.all(r["loop"] == -1)
    # With a larger recency window the same neighbours are recent too; one smaller, old.
    r2 = oracle.kf_loop_update(poses, kf, g, nb, PARAMS, n_recent=2)
    assert np.all(r2["loop"] == K - 3)
    for i in range(3):
        assert same_pose(r["poses"][i], poses[i].astype(np.float64), 1e-7)
        for k in range(K):
            assert same_pose(r["kf_poses"][i, k], kf[i, k].astype(np.float64), 1e-7)


def test_zero_path_length_moves_only_the_current_pose():
    K = 5
    kf = np.stack([ident((1.0, 2.0, 3.0)) for _ in range(K)])[None]
    pose = ident((1.0, 2.0, 3.0))[None]
    g = np.array([[0.1, 0.0, 0.0, 0.0, 0.0, 0.1]])
    r = oracle.kf_loop_update(pose, kf, g, np.array([[0, 4]], np.int32), PARAMS, n_recent=3)
    assert r["loop"][0] == 0
    assert np.array_equal(r["kf_poses"][0], kf[0].astype(np.float64))
    assert same_pose(r["poses"][0], mat_pose(pose_mat(pose[0]) @ expm(twist(g[0]))))
