"""Seeded inputs of the GICP likelihood: voxelised keyframe Gaussians and
per-point scan covariances (the distribution-to-distribution model of the
paper's Sec. III-C.1, with voxel-based correspondences).

Voxel (i, j, k) of a map with origin o and edge vs covers
[o + (i, j, k) vs, o + (i+1, j+1, k+1) vs) and holds 12 FP32 values: the mean
of the points in it (3), their count, their covariance regularised by
reg * I (xx xy xz yy yz zz), and 2 unused.  Voxels with fewer than
`min_count` points are empty (count 0).  A scan point's covariance is that of
its k nearest scan neighbours (itself included), regularised the same way.
"""

import numpy as np

REG = 0.02 ** 2


def voxel_gaussians(points, dims, origin, vs, min_count=5, reg=REG):
    """(nz, ny, nx, 12) FP32 voxel Gaussians of `points` (n, 3)."""
    nx, ny, nz = (int(v) for v in dims)
    pts = np.asarray(points, np.float64)
    idx = np.floor((pts - np.asarray(origin, np.float64)) / vs).astype(np.int64)
    ok = np.all((idx >= 0) & (idx < [nx, ny, nz]), axis=1)
    pts, idx = pts[ok], idx[ok]
    lin = idx[:, 0] + nx * (idx[:, 1] + ny * idx[:, 2])
    order = np.argsort(lin, kind="stable")
    lin, pts = lin[order], pts[order]
    out = np.zeros((nx * ny * nz, 12), np.float32)
    starts = np.flatnonzero(np.r_[True, lin[1:] != lin[:-1]])
    ends = np.r_[starts[1:], len(lin)]
    for s, e in zip(starts, ends):
        n = e - s
        if n < min_count:
            continue
        p = pts[s:e]
        mu = p.mean(axis=0)
        d = p - mu
        C = d.T @ d / n + reg * np.eye(3)
        out[lin[s]] = [mu[0], mu[1], mu[2], n, C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2], C[2, 2], 0, 0]
    return out.reshape(nz, ny, nx, 12)


def point_covariances(points, k=10, reg=REG):
    """(M, 6) FP32 covariances of each point's k nearest neighbours (itself included)."""
    from scipy.spatial import cKDTree
    pts = np.asarray(points, np.float64)
    k = min(k, len(pts))
    _, nb = cKDTree(pts).query(pts, k=k)
    nb = nb.reshape(len(pts), k)
    q = pts[nb]
    d = q - q.mean(axis=1, keepdims=True)
    C = np.einsum("nki,nkj->nij", d, d) / k + reg * np.eye(3)
    return np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]],
                    axis=1).astype(np.float32)
