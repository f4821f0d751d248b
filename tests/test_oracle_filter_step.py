"""Pins for the oracle's whole-frame composition and for its cell-face allowance.

oracle.filter_step chains prediction (Eq. 1), I passes of likelihood, gradient
and step (Sec. III-C, Eq. 7), weighting (Eq. 11), normalisation and systematic
resampling.  It is checked against the same sequence built here from stages
pinned on their own: evaluate_f64 (finite differences, closed forms), the pose
algebra written with scipy's matrix exponential, weights (long double) and
resample (exact rationals).  The face allowance of evaluate(delta=...) is
checked against a brute-force trilinear evaluation of both cells at a face.
"""

import math

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle


def twist(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
    X[:3, 3] = xi[:3]
    return X


def T_of(pose):
    q = np.asarray(pose[3:], np.float64)
    q = q / np.linalg.norm(q)
    T = np.eye(4)
    T[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    T[:3, 3] = pose[:3]
    return T


def pose_of(T):
    x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
    return np.array([T[0, 3], T[1, 3], T[2, 3], w, x, y, z])


def clamp(v, m):
    n = np.linalg.norm(v)
    return v * (m / n) if n > m else v


def composed_frame(c, scan, poses, logw, p, u, policy, dT, delta, post_eval):
    """The frame from pinned stages, pose algebra in 4x4 matrices."""
    N = poses.shape[0]
    T = [T_of(poses[i].astype(np.float64)) @ T_of(dT) @ expm(twist(delta[i].astype(np.float64)))
         for i in range(N)]
    args = (c["grid"], c["dims"], c["origin"], c["h"], p["eps"], scan)
    for _ in range(p["iters"]):
        cur = np.stack([pose_of(Ti) for Ti in T])
        ll, g = oracle.evaluate_f64(*args, cur)
        for i in range(N):
            psi = np.concatenate([clamp(p["alpha_t"] * g[i, :3], p["rho_max"]),
                                  clamp(p["alpha_r"] * g[i, 3:], p["phi_max"])])
            T[i] = T[i] @ expm(twist(psi))
    grad = g
    if post_eval:
        ll, _ = oracle.evaluate_f64(*args, np.stack([pose_of(Ti) for Ti in T]))
    lw, L, ess = oracle.weights(logw, ll, p["beta"])
    fire = policy == oracle.POLICY_ALWAYS or (policy == oracle.POLICY_ESS and ess < 0.5 * N)
    anc = oracle.resample(lw, u)[0] if fire else np.arange(N)
    out_T = [T[a] for a in anc]
    out_w = np.full(N, -math.log(N)) if fire else lw
    return dict(T=out_T, logw=out_w, loglik=ll, grad=grad, anc=anc, lse=L, ess=ess, fire=fire)


def test_filter_step_is_the_composition_of_its_stages(box_room):
    c = box_room
    rng = np.random.default_rng(7)
    N = 40
    scan = c["scan"][::8]
    poses = c["poses"][:N]
    dq = np.array([0.998, 0.02, -0.03, 0.05])
    dT = np.concatenate([[0.3, -0.2, 0.05], dq / np.linalg.norm(dq)])
    delta = (rng.normal(size=(N, 6)) * [0.05, 0.05, 0.05, 0.017, 0.017, 0.017]).astype(np.float32)
    for policy, post_eval, beta, iters in ((oracle.POLICY_ALWAYS, False, 1.0, 3),
                                           (oracle.POLICY_ESS, True, 0.01, 2),
                                           (oracle.POLICY_NEVER, False, 0.05, 1)):
        p = dict(c["params"], iters=iters, beta=beta)
        logw = rng.normal(size=N) * 0.3
        u = 0.37
        got = oracle.filter_step(c["grid"], c["dims"], c["origin"], c["h"], scan, poses, logw, p, u,
                                 policy=policy, dT=dT, delta=delta, post_eval=post_eval)
        ref = composed_frame(c, scan, poses, logw, p, u, policy, dT, delta, post_eval)
        assert got["resampled"] == ref["fire"]
        assert np.array_equal(got["ancestors"], ref["anc"])
        assert np.allclose(got["loglik"], ref["loglik"], rtol=1e-11, atol=0)
        gs = np.abs(ref["grad"]).max()
        assert np.allclose(got["grad"], ref["grad"], rtol=1e-9, atol=1e-9 * gs)
        assert abs(got["lse"] - ref["lse"]) <= 1e-11 * max(1.0, abs(ref["lse"]))
        assert abs(got["ess"] - ref["ess"]) <= 1e-9 * ref["ess"]
        assert np.allclose(got["logw"], ref["logw"], rtol=0, atol=1e-9)
        for k in range(N):
            Tg = T_of(got["poses"][k])
            assert np.allclose(Tg[:3, 3], ref["T"][k][:3, 3], atol=1e-11)
            assert np.allclose(Tg[:3, :3], ref["T"][k][:3, :3], atol=1e-12)


# -- cell-face allowance -----------------------------------------------------

def cell_eval(grid, i0, f, h, eps):
    """ln(G + eps) and its world gradient in cell i0 at fractions f (brute force)."""
    G, dG = 0.0, np.zeros(3)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                v = float(grid[i0[2] + c, i0[1] + b, i0[0] + a])
                w = [(1 - f[0], f[0])[a], (1 - f[1], f[1])[b], (1 - f[2], f[2])[c]]
                s = [2 * a - 1, 2 * b - 1, 2 * c - 1]
                G += v * w[0] * w[1] * w[2]
                dG += v * np.array([s[0] * w[1] * w[2], w[0] * s[1] * w[2], w[0] * w[1] * s[2]])
    return math.log(G + eps), dG / (h * (G + eps))


def test_face_allowance_is_the_largest_change_over_both_cells():
    rng = np.random.default_rng(11)
    n, h, eps = 8, 0.2, 1e-3
    grid = rng.uniform(0, 1, (n, n, n)).astype(np.float32)
    origin = np.zeros(3)
    delta = 1e-3
    # A one-point scan at p with an identity pose: u = p/h - 1/2.
    for axis in range(3):
        u = np.array([3.4, 2.7, 4.2])
        u[axis] = 3.0 + 0.4 * delta            # just above the face u = 3 on this axis
        p = ((u + 0.5) * h).astype(np.float32)[None, :]
        uf = p[0].astype(np.float64) / h - 0.5  # the index coordinate of the FP32 point
        pose = np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32)
        r = oracle.evaluate(grid, (n, n, n), origin, h, eps, p, pose, delta=delta)
        assert r["n_amb"][0] == 1
        i0 = np.floor(uf).astype(int)
        f = uf - i0
        l0, d0 = cell_eval(grid, i0, f, h, eps)
        v = p[0].astype(np.float64)
        amb_l, amb_g = 0.0, np.zeros(6)
        # Positions within delta of the face on either side: lower cell at
        # fractions 1 - delta and 1, upper cell at 0 and delta.
        for off, fr in ((-1, 1 - delta), (-1, 1.0), (0, 0.0), (0, delta)):
            j0, ff = i0.copy(), f.copy()
            j0[axis], ff[axis] = 3 + off, fr
            l, d = cell_eval(grid, j0, ff, h, eps)
            amb_l = max(amb_l, abs(l - l0))
            amb_g = np.maximum(amb_g, np.abs(np.concatenate([d - d0, np.cross(v, d) - np.cross(v, d0)])))
        assert abs(r["loglik"][0] - l0) < 1e-12
        assert abs(r["amb_l"][0] - amb_l) <= 1e-12 * max(1.0, amb_l)
        assert np.allclose(r["amb_g"][0], amb_g, rtol=1e-10, atol=1e-12)
    # Away from every face: no allowance.
    p = ((np.array([3.4, 2.7, 4.2]) + 0.5) * h).astype(np.float32)[None, :]
    r = oracle.evaluate(grid, (n, n, n), origin, h, eps, p, np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32),
                        delta=delta)
    assert r["n_amb"][0] == 0 and r["amb_l"][0] == 0 and np.all(r["amb_g"][0] == 0)
