"""Rotation helpers for building inputs (scene poses, sensor frames, noise).

These only place sensors and particles in the synthetic world; the filter's
own SE(3) arithmetic lives separately in the oracle and in the HIP kernels.
Quaternions are Hamilton, ordered (w, x, y, z), active body-to-world.
"""

import numpy as np


def quat_from_axis_angle(phi):
    """Unit quaternion(s) for rotation vector(s) ``phi`` (..., 3)."""
    phi = np.asarray(phi, dtype=np.float64)
    th = np.linalg.norm(phi, axis=-1, keepdims=True)
    half = 0.5 * th
    # sin(th/2)/th, written with np.sinc to stay exact at th == 0.
    s = 0.5 * np.sinc(half / np.pi)
    return np.concatenate([np.cos(half), s * phi], axis=-1)


def quat_mul(a, b):
    """Hamilton product a (x) b, broadcasting over leading axes."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quat_to_matrix(q):
    """Rotation matrix (..., 3, 3) of unit quaternion(s) (..., 4)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(q, -1, 0)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], axis=-2)


def quat_yaw(yaw):
    """Quaternion of a rotation by ``yaw`` about the world z axis."""
    yaw = np.asarray(yaw, dtype=np.float64)
    z = np.zeros_like(yaw)
    return np.stack([np.cos(0.5 * yaw), z, z, np.sin(0.5 * yaw)], axis=-1)


def pose_matrix(t, q):
    """4x4 homogeneous matrix of translation t and quaternion q."""
    T = np.eye(4)
    T[:3, :3] = quat_to_matrix(q)
    T[:3, 3] = t
    return T


def matrix_to_pose(T):
    """(t, q) of a 4x4 rigid transform, with q.w >= 0 (Shepperd's method)."""
    R = T[:3, :3]
    tr = np.trace(R)
    if tr > 0:
        s = 2.0 * np.sqrt(tr + 1.0)
        q = np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s,
                      (R[1, 0] - R[0, 1]) / s])
    else:
        i = int(np.argmax(np.diag(R)))
        j, k = (i + 1) % 3, (i + 2) % 3
        s = 2.0 * np.sqrt(1.0 + R[i, i] - R[j, j] - R[k, k])
        q = np.empty(4)
        q[0] = (R[k, j] - R[j, k]) / s
        q[1 + i] = 0.25 * s
        q[1 + j] = (R[j, i] + R[i, j]) / s
        q[1 + k] = (R[k, i] + R[i, k]) / s
    if q[0] < 0:
        q = -q
    return T[:3, 3].copy(), q / np.linalg.norm(q)


def rotvec_from_matrix(R):
    """Rotation vector of a rotation matrix (angle < pi)."""
    c = np.clip(0.5 * (np.trace(R) - 1.0), -1.0, 1.0)
    th = np.arccos(c)
    w = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-12:
        return 0.5 * w
    return th / (2.0 * np.sin(th)) * w
