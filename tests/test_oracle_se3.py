"""Pins for the oracle's SE(3) arithmetic (Eq. 1 and Eq. 7 of the paper).

The reference points are independent of the oracle: scipy's Pade
scaling-and-squaring matrix exponential of the 4x4 twist, and scipy's
rotation conversions.
"""

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle


def hat(phi):
    return np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])


def twist(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = hat(xi[3:])
    X[:3, 3] = xi[:3]
    return X


def quat_of(Rm):
    x, y, z, w = Rotation.from_matrix(Rm).as_quat()
    return np.array([w, x, y, z])


ANGLES = [0.0, 1e-12, 1e-9, 1e-6, 1e-3, 0.05, 0.0999999, 0.1, 0.1000001, 0.7, 2.0, 3.1]


@pytest.mark.parametrize("ang", ANGLES)
def test_exp_matches_matrix_exponential(ang):
    rng = np.random.default_rng(int(ang * 1e6) + 7)
    for _ in range(5):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        xi = np.concatenate([rng.normal(size=3) * 3.0, axis * ang])
        T = oracle.se3_exp(xi)
        assert np.allclose(T, expm(twist(xi)), rtol=0, atol=1e-12)


def test_rotation_is_orthonormal():
    rng = np.random.default_rng(3)
    for _ in range(100):
        q = rng.normal(size=4)
        R = oracle.quat_to_rot(q)
        assert np.allclose(R.T @ R, np.eye(3), atol=2e-15)
        assert abs(np.linalg.det(R) - 1.0) < 4e-15  # a few ulps of the determinant itself
        # Same rotation as scipy's (Hamilton, scalar-last in scipy).
        q = q / np.linalg.norm(q)
        Rs = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.allclose(R, Rs, atol=1e-15)


@pytest.mark.parametrize("ang", [0.0, 1e-9, 1e-4, 0.0999, 0.1001, 1.0, 3.0, np.pi - 1e-6])
def test_log_exp_round_trip(ang):
    rng = np.random.default_rng(11)
    for _ in range(5):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        xi = np.concatenate([rng.normal(size=3) * 2.0, axis * ang])
        xi2 = oracle.se3_log(oracle.se3_exp(xi))
        assert np.allclose(xi2, xi, atol=1e-9 if ang > 3 else 1e-12)
        T = expm(twist(xi))
        assert np.allclose(oracle.se3_exp(oracle.se3_log(T)), T, atol=1e-12)


def test_small_angle_branch_is_continuous():
    # The V-matrix switches from a Taylor series to the closed form at 0.1 rad.
    axis = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    rho = np.array([1.0, 2.0, -3.0])
    lo = oracle.se3_exp(np.concatenate([rho, axis * (0.1 - 1e-12)]))
    hi = oracle.se3_exp(np.concatenate([rho, axis * (0.1 + 1e-12)]))
    assert np.abs(lo - hi).max() < 1e-11


def test_pose_right_exp_matches_matrix_product():
    rng = np.random.default_rng(5)
    for _ in range(50):
        t = rng.normal(size=3) * 30
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        psi = np.concatenate([rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.2])
        out = oracle.pose_right_exp(np.concatenate([t, q]), psi)
        T = np.eye(4)
        T[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        T[:3, 3] = t
        Tn = T @ expm(twist(psi))
        assert np.allclose(out[:3], Tn[:3, 3], atol=1e-12)
        Rn = Rotation.from_quat([out[4], out[5], out[6], out[3]]).as_matrix()
        assert np.allclose(Rn, Tn[:3, :3], atol=1e-13)
        assert abs(np.linalg.norm(out[3:]) - 1.0) < 1e-15


def test_exp_of_zero_is_identity():
    pose = np.array([1.0, -2.0, 3.0, 0.5, 0.5, 0.5, 0.5])
    out = oracle.pose_right_exp(pose, np.zeros(6))
    assert np.array_equal(out[:3], pose[:3])
    assert np.allclose(out[3:], pose[3:], atol=1e-16)
