"""Central finite differences pin the oracle's analytic gradient.

For every (particle, point) pair the oracle's per-point gradient is compared
with (l(T Exp(+h e_c)) - l(T Exp(-h e_c))) / 2h, h = 1e-6 (m and rad), at rel
1e-6.  The perturbed poses come from scipy's matrix exponential, not from the
oracle.  The trilinear interpolant has kinks on cell faces, so a point whose
two stencil positions fall in different cells is excluded and counted.
"""

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle

STEP = 1e-6


def twist(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
    X[:3, 3] = xi[:3]
    return X


def pose_to_T(pose):
    T = np.eye(4)
    q = pose[3:] / np.linalg.norm(pose[3:])
    T[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    T[:3, 3] = pose[:3]
    return T


def T_to_pose(T):
    x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
    return np.array([T[0, 3], T[1, 3], T[2, 3], w, x, y, z])


def cell_of(T, p, origin, h):
    x = T[:3, :3] @ p + T[:3, 3]
    u = (x - np.asarray(origin)) / h - 0.5
    return np.floor(u)


def check_fd(cfg, n_particles, n_points, eps, seed):
    rng = np.random.default_rng(seed)
    grid, dims, origin, h = cfg["grid"], cfg["dims"], cfg["origin"], cfg["h"]
    idx_p = rng.choice(cfg["poses"].shape[0], n_particles, replace=False)
    idx_j = rng.choice(cfg["scan"].shape[0], n_points, replace=False)
    excluded = used = 0
    for i in idx_p:
        pose = cfg["poses"][i].astype(np.float64)
        pose[3:] /= np.linalg.norm(pose[3:])
        T = pose_to_T(pose)
        stencil = []
        for c in range(6):
            for s in (+1, -1):
                xi = np.zeros(6)
                xi[c] = s * STEP
                stencil.append(T @ expm(twist(xi)))
        poses_fd = np.array([T_to_pose(Ts) for Ts in stencil])
        sum_fd = np.zeros(6)
        sum_an = np.zeros(6)
        for j in idx_j:
            p = cfg["scan"][j:j + 1]
            pj = p[0].astype(np.float64)
            ll, _ = oracle.evaluate_f64(grid, dims, origin, h, eps, p, poses_fd)
            _, g = oracle.evaluate_f64(grid, dims, origin, h, eps, p, pose[None, :])
            for c in range(6):
                cp = cell_of(stencil[2 * c], pj, origin, h)
                cm = cell_of(stencil[2 * c + 1], pj, origin, h)
                if not np.array_equal(cp, cm):
                    excluded += 1
                    continue
                fd = (ll[2 * c] - ll[2 * c + 1]) / (2 * STEP)
                an = g[0, c]
                used += 1
                assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (i, j, c, fd, an)
                sum_fd[c] += fd
                sum_an[c] += an
        assert np.allclose(sum_fd, sum_an, rtol=1e-6, atol=1e-6)
    return used, excluded


def test_gradient_matches_central_differences_box_room(box_room):
    used, excluded = check_fd(box_room, 6, 96, box_room["params"]["eps"], 0)
    assert used > 3000
    assert excluded < 0.01 * used


def test_gradient_matches_central_differences_gaussian_source():
    n = (40, 40, 40)
    c = (np.arange(40) + 0.5) * 0.2
    q = np.array([4.1, 3.9, 4.3])
    G = (np.exp(-(c[None, None, :] - q[0]) ** 2 / 0.08) * np.exp(-(c[None, :, None] - q[1]) ** 2 / 0.08)
         * np.exp(-(c[:, None, None] - q[2]) ** 2 / 0.08)).astype(np.float32)
    rng = np.random.default_rng(9)
    scan = (rng.normal(size=(64, 3)) * 0.4).astype(np.float32)
    quat = rng.normal(size=(4, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    poses = np.column_stack([q + rng.normal(size=(4, 3)) * 0.2, quat]).astype(np.float32)
    cfg = dict(grid=G, dims=n, origin=(0, 0, 0), h=0.2, poses=poses, scan=scan)
    used, excluded = check_fd(cfg, 4, 64, 1e-3, 1)
    assert used > 1400
