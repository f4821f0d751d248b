"""Pins for the oracle's grid likelihood and its gradient.

Each check compares against something fixed by the mathematics rather than by
the oracle's own code:

* trilinear interpolation reproduces any trilinear polynomial exactly, so on a
  grid filled with one the likelihood and gradient are closed forms;
* a grid sampled from an isotropic Gaussian is separable, so its trilinear
  interpolant is a product of three 1-D linear interpolants;
* a point on a voxel centre returns the stored sample;
* a floor-only map has a gradient along the world z axis only;
* points outside the grid contribute exactly ln(eps) (or nothing);
* the point transform uses scipy's rotation for the expected index coordinates.
"""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle

H = 0.2
EPS = 1e-3


def rot(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def poly_grid(n, coef):
    """Grid of the trilinear polynomial P(x,y,z) at integer index coordinates."""
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    c = coef
    P = (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z
         + c[7] * x * y * z)
    return P.astype(np.float64)


def poly_and_grad(u, c):
    x, y, z = u
    P = c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z + c[7] * x * y * z
    dP = np.array([c[1] + c[4] * y + c[5] * z + c[7] * y * z,
                   c[2] + c[4] * x + c[6] * z + c[7] * x * z,
                   c[3] + c[5] * x + c[6] * y + c[7] * x * y])
    return P, dP


def test_trilinear_polynomial_is_reproduced_exactly():
    n = (7, 6, 5)
    coef = [40, 3, 5, 7, 1, 2, 1, 1]            # integers: every sample is exact in FP32
    G = poly_grid(n, coef)
    assert G.max() < 2 ** 24
    origin = np.array([-1.0, 2.0, 0.5])
    rng = np.random.default_rng(0)
    pose = np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32)
    for _ in range(200):
        u = rng.uniform(0, np.array(n) - 1 - 1e-9)
        # World point whose index coordinate is u: x = o + (u + 1/2) h.
        p = (origin + (u + 0.5) * H).astype(np.float32)
        u_exact = (p.astype(np.float64) - origin) / H - 0.5
        r = oracle.evaluate(G, n, origin, H, EPS, p[None, :], pose)
        P, dP = poly_and_grad(u_exact, coef)
        assert r["loglik"][0] == pytest.approx(math.log(P + EPS), rel=1e-14)
        grad_x = dP / (H * (P + EPS))
        assert np.allclose(r["grad"][0, :3], grad_x, rtol=1e-12, atol=1e-14)
        assert np.allclose(r["grad"][0, 3:], np.cross(p.astype(np.float64), grad_x), rtol=1e-11,
                           atol=1e-12)


def gaussian_grid(n, origin, q, sigma):
    c = [origin[a] + (np.arange(n[a]) + 0.5) * H for a in range(3)]
    g1 = [np.exp(-(c[a] - q[a]) ** 2 / (2 * sigma ** 2)) for a in range(3)]
    G = g1[2][:, None, None] * g1[1][None, :, None] * g1[0][None, None, :]
    return G.astype(np.float32), g1


def test_single_source_separable_closed_form():
    """G(c) = exp(-|c - q|^2 / 2 sigma^2) factorises over axes, and so does its
    trilinear interpolant: G(u) = prod_a [(1 - f_a) g_a(i_a) + f_a g_a(i_a + 1)]."""
    n = (24, 20, 16)
    origin = np.array([1.0, -2.0, 0.0])
    q = origin + np.array([2.3, 1.9, 1.7])
    sigma = 0.25
    G, g1 = gaussian_grid(n, origin, q, sigma)
    rng = np.random.default_rng(1)
    for _ in range(100):
        t = rng.normal(size=3) * 0.1 + q
        quat = rng.normal(size=4)
        quat /= np.linalg.norm(quat)
        pose = np.concatenate([t, quat]).astype(np.float32)
        p = (rng.normal(size=3) * 0.3).astype(np.float32)
        R = rot(pose[3:].astype(np.float64))
        x = R @ p.astype(np.float64) + pose[:3].astype(np.float64)
        u = (x - origin) / H - 0.5
        i0 = np.floor(u).astype(int)
        f = u - i0
        lerp = [(1 - f[a]) * float(g1[a][i0[a]]) + f[a] * float(g1[a][i0[a] + 1]) for a in range(3)]
        dlerp = [float(g1[a][i0[a] + 1]) - float(g1[a][i0[a]]) for a in range(3)]
        Gu = lerp[0] * lerp[1] * lerp[2]
        dG = np.array([dlerp[0] * lerp[1] * lerp[2], lerp[0] * dlerp[1] * lerp[2],
                       lerp[0] * lerp[1] * dlerp[2]])
        r = oracle.evaluate(G, n, origin, H, EPS, p[None, :], pose[None, :])
        # The stored grid is the FP32 rounding of the separable product.
        assert r["loglik"][0] == pytest.approx(math.log(Gu + EPS), rel=2e-7, abs=2e-7)
        grad_x = dG / (H * (Gu + EPS))
        scale = np.abs(grad_x).max() + 1e-3
        assert np.abs(r["grad"][0, :3] - R.T @ grad_x).max() < 2e-6 * scale
        g_phi = R.T @ np.cross(R @ p.astype(np.float64), grad_x)
        assert np.abs(r["grad"][0, 3:] - g_phi).max() < 2e-6 * scale * (1 + np.linalg.norm(p))


def test_voxel_centre_returns_stored_sample():
    n = (9, 8, 7)
    rng = np.random.default_rng(2)
    G = rng.uniform(0, 1, (n[2], n[1], n[0])).astype(np.float32)
    origin = np.array([0.3, 0.1, -0.4])
    pose = np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32)
    for _ in range(50):
        i = [int(rng.integers(0, n[a] - 1)) for a in range(3)]
        # Power-of-two spacing keeps the voxel centre exact in FP32 and FP64.
        h = 0.25
        org = np.round(origin * 4) / 4
        p = (org + (np.array(i) + 0.5) * h).astype(np.float32)
        r = oracle.evaluate(G, n, org, h, EPS, p[None, :], pose)
        assert r["loglik"][0] == math.log(float(G[i[2], i[1], i[0]]) + EPS)


def test_floor_only_map_has_vertical_gradient():
    n = (32, 32, 32)
    c = (np.arange(32) + 0.5) * H
    gz = np.exp(-(c - 2.0) ** 2 / (2 * 0.1 ** 2))
    G = np.broadcast_to(gz[:, None, None], (32, 32, 32)).astype(np.float32)
    rng = np.random.default_rng(3)
    scan = (rng.normal(size=(300, 3)) * 1.5).astype(np.float32)
    quat = rng.normal(size=(20, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    t = np.column_stack([rng.uniform(2, 4, (20, 2)), rng.uniform(1.8, 2.2, 20)])
    poses = np.column_stack([t, quat]).astype(np.float32)
    r = oracle.evaluate(G, n, (0, 0, 0), H, EPS, scan, poses)
    for k in range(20):
        R = rot(poses[k, 3:].astype(np.float64))
        gw = R @ r["grad"][k, :3]             # world-frame translation gradient
        rw = R @ r["grad"][k, 3:]             # world-frame rotation gradient
        s = np.abs(r["gabs"][k]).max()
        assert abs(gw[0]) < 1e-12 * s and abs(gw[1]) < 1e-12 * s
        assert abs(rw[2]) < 1e-12 * s         # no torque about the world vertical
        assert np.abs(gw[2]) > 0


def test_out_of_bounds_and_nan_points():
    n = (8, 8, 8)
    G = np.full((8, 8, 8), 0.5, np.float32)
    pose = np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32)
    # Index coordinate u = x/h - 1/2: valid range is [0, 7).
    pts = np.array([[-0.2, 0.5, 0.5], [1.5, 0.5, 0.5], [0.5, 0.5, 5.0], [np.nan, 0.5, 0.5],
                    [0.5, np.inf, 0.5]], np.float32)
    for k in range(len(pts)):
        r = oracle.evaluate(G, n, (0, 0, 0), H, EPS, pts[k:k + 1], pose)
        assert r["loglik"][0] == math.log(np.float64(np.float32(EPS))) or \
            r["loglik"][0] == math.log(EPS)
        assert np.all(r["grad"][0] == 0.0)
        r = oracle.evaluate(G, n, (0, 0, 0), H, EPS, pts[k:k + 1], pose, oob_skip=True)
        assert r["loglik"][0] == 0.0 and np.all(r["grad"][0] == 0.0)
    # Boundary: u = 0 is inside, u = n - 1 is outside.
    inside = np.array([[0.1, 0.1, 0.1]], np.float32)     # u = 0 (0.1/0.2 - 0.5)
    r = oracle.evaluate(G, n, (0, 0, 0), H, EPS, inside, pose)
    assert r["loglik"][0] == pytest.approx(math.log(0.5 + EPS), rel=1e-12)


def test_point_transform_uses_the_pose():
    """l of a scan under pose T equals l of the world points under the identity."""
    from synth import configs
    c = configs.box_room(N=8)
    eps = c["params"]["eps"]
    rng = np.random.default_rng(4)
    scan = c["scan"][:64].astype(np.float64)
    for k in range(8):
        pose = c["poses"][k].astype(np.float64)
        R = rot(pose[3:] / np.linalg.norm(pose[3:]))
        world = scan @ R.T + pose[:3]
        a = oracle.evaluate(c["grid"], c["dims"], c["origin"], c["h"], eps, c["scan"][:64],
                            c["poses"][k:k + 1])
        b = oracle.evaluate_f64(c["grid"], c["dims"], c["origin"], c["h"], eps,
                                world.astype(np.float32), np.array([[0, 0, 0, 1, 0, 0, 0.0]]))
        # world points rounded to FP32 move u by <1e-6 voxel; G is Lipschitz.
        assert a["loglik"][0] == pytest.approx(b[0][0], rel=1e-4)
    del rng
