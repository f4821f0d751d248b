"""Pins for the gradient-guided pose step (Eq. 7) and the prediction (Eq. 1)."""

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle


def twist(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
    X[:3, 3] = xi[:3]
    return X


def pose_to_T(pose):
    T = np.eye(4)
    q = np.asarray(pose[3:], np.float64)
    q = q / np.linalg.norm(q)
    T[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    T[:3, 3] = pose[:3]
    return T


def test_zero_gradient_leaves_pose():
    rng = np.random.default_rng(0)
    poses = np.column_stack([rng.normal(size=(10, 3)), rng.normal(size=(10, 4))]).astype(np.float32)
    out = oracle.step(poses, np.zeros((10, 6)), 1e-3, 1e-4, 0.1, 0.01)
    assert np.array_equal(out[:, :3], poses[:, :3].astype(np.float64))
    qn = poses[:, 3:].astype(np.float64)
    qn /= np.linalg.norm(qn, axis=1, keepdims=True)
    assert np.allclose(out[:, 3:], qn, atol=1e-16)


def test_step_is_T_exp_psi_with_clamp():
    rng = np.random.default_rng(1)
    N = 200
    poses = np.column_stack([rng.normal(size=(N, 3)) * 20, rng.normal(size=(N, 4))]).astype(np.float32)
    g = rng.normal(size=(N, 6)) * np.array([300, 300, 300, 5000, 5000, 5000.0])
    at, ar, rmax, pmax = 2e-4, 3e-6, 0.1, 0.012
    out = oracle.step(poses, g, at, ar, rmax, pmax)
    n_clamped = 0
    for i in range(N):
        psi = np.concatenate([at * g[i, :3], ar * g[i, 3:]])
        nr, npn = np.linalg.norm(psi[:3]), np.linalg.norm(psi[3:])
        if nr > rmax:
            psi[:3] *= rmax / nr
            n_clamped += 1
        if npn > pmax:
            psi[3:] *= pmax / npn
        Tn = pose_to_T(poses[i].astype(np.float64)) @ expm(twist(psi))
        assert np.allclose(out[i, :3], Tn[:3, 3], atol=1e-12)
        assert np.allclose(pose_to_T(out[i])[:3, :3], Tn[:3, :3], atol=1e-13)
    assert 0 < n_clamped < N


def test_clamp_preserves_direction_and_bounds_norm():
    pose = np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32)
    g = np.array([[3.0, -4.0, 12.0, 0.0, 0.0, 0.0]])
    out = oracle.step(pose, g, 1.0, 1.0, 0.5, 1.0)
    d = out[0, :3]
    assert abs(np.linalg.norm(d) - 0.5) < 1e-15
    assert np.allclose(d / np.linalg.norm(d), g[0, :3] / 13.0, atol=1e-15)
    g = np.array([[0.0, 0.0, 0.0, 0.0, 0.0, 2.0]])
    out = oracle.step(pose, g, 1.0, 1.0, 0.5, 0.25)
    # A pure yaw of 0.25 rad.
    assert np.allclose(out[0, 3:], [np.cos(0.125), 0, 0, np.sin(0.125)], atol=1e-15)


def test_small_step_increases_likelihood(box_room):
    """Ascent: a small step along g raises l, consistent with the gradient's sign."""
    c = box_room
    eps = c["params"]["eps"]
    sub = c["poses"][:64]
    r0 = oracle.evaluate(c["grid"], c["dims"], c["origin"], c["h"], eps, c["scan"], sub)
    moved = oracle.step(sub, r0["grad"], 1e-7, 1e-9, 1.0, 1.0)
    l1, _ = oracle.evaluate_f64(c["grid"], c["dims"], c["origin"], c["h"], eps, c["scan"], moved)
    l0, _ = oracle.evaluate_f64(c["grid"], c["dims"], c["origin"], c["h"], eps, c["scan"],
                                sub.astype(np.float64))
    gn = np.linalg.norm(r0["grad"], axis=1)
    ok = gn > 1.0
    assert ok.sum() > 50
    assert np.mean(l1[ok] > l0[ok]) > 0.95


def test_prediction_is_T_dT_exp_delta():
    rng = np.random.default_rng(2)
    N = 100
    poses = np.column_stack([rng.normal(size=(N, 3)) * 30, rng.normal(size=(N, 4))]).astype(np.float32)
    dq = rng.normal(size=4)
    dq /= np.linalg.norm(dq)
    dT = np.concatenate([rng.normal(size=3), dq])
    delta = (rng.normal(size=(N, 6)) * 0.05).astype(np.float32)
    out = oracle.predict(poses, dT, delta)
    out0 = oracle.predict(poses, dT, None)
    for i in range(N):
        Tn = pose_to_T(poses[i].astype(np.float64)) @ pose_to_T(dT) @ expm(twist(delta[i].astype(np.float64)))
        assert np.allclose(out[i, :3], Tn[:3, 3], atol=1e-12)
        assert np.allclose(pose_to_T(out[i])[:3, :3], Tn[:3, :3], atol=1e-13)
        T0 = pose_to_T(poses[i].astype(np.float64)) @ pose_to_T(dT)
        assert np.allclose(out0[i, :3], T0[:3, 3], atol=1e-12)
