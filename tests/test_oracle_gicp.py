"""Pins for the oracle's GICP likelihood and Gauss-Newton step (Eq. 2-7).

References independent of the oracle: the Jacobian of the residual by central
finite differences of poses built with scipy's matrix exponential, numpy's
dense solver for the 6x6 system, invariance of every output to a rigid
motion applied to the whole scene, and convergence of the step on a
well-conditioned synthetic problem.
"""

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle
from synth import gicp

from test_oracle_se3 import twist


def pose_row(T):
    x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
    return np.array([*T[:3, 3], w, x, y, z], np.float32)


def pose_mat(p):
    T = np.eye(4)
    q = np.asarray(p[3:], np.float64)
    q /= np.linalg.norm(q)
    T[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    T[:3, 3] = p[:3]
    return T


def box_points(rng, n=6000, lo=-3.8, hi=3.8):
    """Points on the six faces of a box (well-conditioned for registration), the faces
    away from voxel boundaries."""
    f = rng.integers(0, 6, n)
    p = rng.uniform(lo, hi, (n, 3))
    ax = f // 2
    p[np.arange(n), ax] = np.where(f % 2 == 0, lo, hi)
    return p


def make_problem(seed=1, n_scan=400, vs=0.5, dims=(24, 24, 24)):
    rng = np.random.default_rng(seed)
    world = box_points(rng, 20000)
    origin = np.full(3, -6.0)
    vox = gicp.voxel_gaussians(world, dims, origin, vs)
    scan = box_points(rng, n_scan) + rng.normal(0, 0.005, (n_scan, 3))
    cov = gicp.point_covariances(scan)
    return vox, origin, vs, dims, scan.astype(np.float32), cov


def test_jacobian_against_finite_differences():
    vox, origin, vs, dims, scan, cov = make_problem(seed=2, n_scan=1)
    # One point, one keyframe at the identity, a particle slightly off.
    T = expm(twist(np.array([0.03, -0.02, 0.01, 0.01, -0.02, 0.015])))
    pose = pose_row(T)
    kf = pose_row(np.eye(4))[None, None]
    r = oracle.gicp_evaluate(vox, dims, origin[None], vs, scan, cov, pose[None], kf, n_nb=1)
    assert r["n_corr"][0] == 1
    # The voxel Gaussian of the point, located independently.
    Tp = pose_mat(pose)
    x = Tp[:3, :3] @ scan[0].astype(np.float64) + Tp[:3, 3]
    i = np.floor((x - origin) / vs).astype(int)
    v = vox[i[2], i[1], i[0]].astype(np.float64)
    mu_v = v[:3]
    Sv = np.array([[v[4], v[5], v[6]], [v[5], v[7], v[8]], [v[6], v[8], v[9]]])
    c = cov[0].astype(np.float64)
    Ss = np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])
    R = Tp[:3, :3]
    Om = np.linalg.inv(Sv + R @ Ss @ R.T)

    def e_of(xi):
        Tx = Tp @ expm(twist(xi))
        return mu_v - (Tx[:3, :3] @ scan[0].astype(np.float64) + Tx[:3, 3])

    h = 1e-6
    J = np.stack([(e_of(h * np.eye(6)[c]) - e_of(-h * np.eye(6)[c])) / (2 * h) for c in range(6)], axis=1)
    e = e_of(np.zeros(6))
    H_fd = J.T @ Om @ J
    b_fd = J.T @ Om @ e
    assert abs(r["loglik"][0] + e @ Om @ e) < 1e-10
    iu = np.triu_indices(6)
    assert np.allclose(r["H"][0], H_fd[iu], rtol=1e-6, atol=1e-8 * np.abs(H_fd).max())
    assert np.allclose(r["b"][0], b_fd, rtol=1e-6, atol=1e-8 * np.abs(b_fd).max())


def test_rigid_motion_of_the_scene_changes_nothing():
    vox, origin, vs, dims, scan, cov = make_problem(seed=3, n_scan=100)
    rng = np.random.default_rng(3)
    N, K = 6, 3
    kf_T = [expm(twist(np.r_[rng.normal(0, 0.2, 3), rng.normal(0, 0.05, 3)])) for _ in range(K)]
    poses_T = [expm(twist(np.r_[rng.normal(0, 0.1, 3), rng.normal(0, 0.03, 3)])) for _ in range(N)]
    G = expm(twist(np.array([30.0, -12.0, 4.0, 0.3, -0.5, 1.1])))
    vox_k = np.stack([vox] * K)
    org = np.stack([origin] * K)

    def run(left):
        poses = np.stack([pose_row(left @ T) for T in poses_T])
        kfs = np.stack([np.stack([pose_row(left @ T) for T in kf_T])] * N)
        # Every keyframe is a neighbour, so the FP32 rounding of the moved poses
        # cannot change the neighbour set; points within 3e-5 voxel of a face may
        # change voxel, so particles with such points are left out.
        return oracle.gicp_evaluate(vox_k, dims, org, vs, scan, cov, poses, kfs, n_nb=K, delta=3e-5)

    a, b = run(np.eye(4)), run(G)
    keep = (a["n_amb"] == 0) & (b["n_amb"] == 0)
    assert keep.sum() >= N // 2
    assert np.array_equal(a["n_corr"][keep], b["n_corr"][keep])
    assert np.all(a["n_corr"] > 0)
    assert np.allclose(a["loglik"][keep], b["loglik"][keep], rtol=1e-5, atol=1e-6)
    assert np.allclose(a["H"][keep], b["H"][keep], rtol=1e-5, atol=1e-6 * np.abs(a["H"]).max())
    assert np.allclose(a["b"][keep], b["b"][keep], rtol=1e-5, atol=1e-5 * np.abs(a["b"]).max())
    assert np.all(a["loglik"] <= 0.0)


def test_gn_solve_matches_dense_solver():
    rng = np.random.default_rng(4)
    N = 50
    iu = np.triu_indices(6)
    Hs, bs = [], []
    for _ in range(N):
        A = rng.normal(size=(6, 6))
        H = A @ A.T + 0.5 * np.eye(6)
        Hs.append(H[iu])
        bs.append(rng.normal(size=6) * 0.01)
    Hs, bs = np.array(Hs), np.array(bs)
    poses = np.tile(np.array([1.0, 2.0, 3.0, 1, 0, 0, 0], np.float32), (N, 1))
    out, psi = oracle.gn_step(poses, Hs, bs, rho_max=10.0, phi_max=10.0)
    for i in range(N):
        H = np.zeros((6, 6))
        H[iu] = Hs[i]
        H = H + np.triu(H, 1).T
        assert np.allclose(psi[i], np.linalg.solve(H, -bs[i]), rtol=1e-10, atol=1e-13)
        assert np.allclose(pose_mat(out[i]), pose_mat(poses[i]) @ expm(twist(psi[i])), atol=1e-12)


def test_gn_step_converges_on_a_box():
    vox, origin, vs, dims, scan, cov = make_problem(seed=5, n_scan=800)
    xi0 = np.array([0.12, -0.08, 0.05, 0.02, -0.015, 0.03])
    pose = pose_row(expm(twist(xi0)))[None]
    kf = pose_row(np.eye(4))[None, None]
    err = [np.linalg.norm(xi0)]
    ll = []
    for _ in range(4):
        r = oracle.gicp_evaluate(vox, dims, origin[None], vs, scan, cov, pose, kf, n_nb=1)
        ll.append(r["loglik"][0])
        new, psi = oracle.gn_step(pose, r["H"], r["b"], rho_max=1.0, phi_max=1.0)
        pose = new.astype(np.float32)
        Tp = pose_mat(pose[0])
        err.append(np.linalg.norm(np.r_[Tp[:3, 3], Rotation.from_matrix(Tp[:3, :3]).as_rotvec()]))
    assert err[-1] < 0.2 * err[0], err
    assert ll[-1] > ll[0]


def test_no_correspondence_gives_nothing():
    vox, origin, vs, dims, scan, cov = make_problem(seed=6)
    far = pose_row(expm(twist(np.array([500.0, 0, 0, 0, 0, 0]))))[None]
    kf = pose_row(np.eye(4))[None, None]
    r = oracle.gicp_evaluate(vox, dims, origin[None], vs, scan, cov, far, kf, n_nb=1)
    assert r["n_corr"][0] == 0 and r["loglik"][0] == 0.0
    assert np.all(r["H"] == 0) and np.all(r["b"] == 0)
    out, psi = oracle.gn_step(far, r["H"], r["b"], 1.0, 1.0)
    assert np.all(psi == 0) and np.allclose(out[0], far[0].astype(np.float64), atol=1e-5)
