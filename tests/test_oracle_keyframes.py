"""Pins for the keyframe-map likelihood: the sum over neighbour keyframes (Eq. 2)
of the grid log-likelihood under the relative pose T_k^-1 T (Eq. 4).

References: the single-grid likelihood at the relative pose composed with
scipy matrices, a stable argsort for the neighbour choice, and additivity
over neighbours.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


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


def make_problem(seed, K=6, N=5, M=80, n=24):
    rng = np.random.default_rng(seed)
    h = 0.2
    dims = (n, n, n)
    grids = rng.uniform(0, 1, (K, n, n, n)).astype(np.float32)
    origins = np.full((K, 3), -0.5 * n * h)
    scan = (rng.normal(size=(M, 3)) * 0.8).astype(np.float32)
    poses = np.column_stack([rng.normal(size=(N, 3)) * 2, rng.normal(size=(N, 4))]).astype(np.float32)
    kf = np.column_stack([rng.normal(size=(N * K, 3)) * 2, rng.normal(size=(N * K, 4))])
    kf = kf.reshape(N, K, 7).astype(np.float32)
    return dict(grids=grids, dims=dims, origins=origins, h=h, scan=scan, poses=poses, kf=kf)


def test_single_neighbour_is_grid_eval_at_relative_pose():
    P = make_problem(0)
    eps = 1e-3
    r = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], eps, P["scan"], P["poses"],
                           P["kf"], n_nb=1)
    for i in range(P["poses"].shape[0]):
        k = r["neighbors"][i, 0]
        Trel = np.linalg.inv(T_of(P["kf"][i, k])) @ T_of(P["poses"][i])
        ll, g = oracle.evaluate_f64(P["grids"][k], P["dims"], P["origins"][k], P["h"], eps, P["scan"],
                                    pose_of(Trel)[None, :])
        assert abs(r["loglik"][i] - ll[0]) < 1e-9 * abs(ll[0])
        assert np.allclose(r["grad"][i], g[0], rtol=1e-8, atol=1e-8 * np.abs(g[0]).max())


def test_neighbours_are_nearest_by_translation_with_stable_ties():
    P = make_problem(1, K=10, N=40)
    # Force exact distance ties: duplicate translations of keyframes 2 and 7.
    P["kf"][:, 7, :3] = P["kf"][:, 2, :3]
    r = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], 1e-3, P["scan"][:4],
                           P["poses"], P["kf"], n_nb=4)
    for i in range(40):
        # Sec. III-C.1: nearest by translation distance; exact ties to the smaller index.
        dd = P["poses"][i, :3].astype(np.float64)[None, :] - P["kf"][i, :, :3].astype(np.float64)
        d2 = np.einsum("ka,ka->k", dd, dd)
        order = np.argsort(d2, kind="stable")
        assert list(r["neighbors"][i]) == list(order[:4])
        # The margin is the smallest relative gap between consecutive ranks 0..4
        # over pairs of distinct translations.
        gaps = [(d2[order[s + 1]] - d2[order[s]]) / d2[order[s + 1]] for s in range(4)
                if not np.array_equal(P["kf"][i, order[s], :3], P["kf"][i, order[s + 1], :3])]
        assert r["nb_margin"][i] == pytest.approx(min(gaps), rel=1e-9, abs=1e-18)


def test_neighbour_margin_flags_near_ties_and_forced_choice():
    P = make_problem(4, K=6, N=3)
    # Keyframe 5 is keyframe 1 moved by one FP32 ulp along x, away from the
    # particle: its squared distance is larger by a relative gap of about 1e-7.
    kx = P["kf"][0, 1, 0]
    away = np.float32(np.inf) if kx > P["poses"][0, 0] else np.float32(-np.inf)
    P["kf"][0, 5, :3] = P["kf"][0, 1, :3]
    P["kf"][0, 5, 0] = np.nextafter(kx, away)
    r = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], 1e-3, P["scan"][:8],
                           P["poses"], P["kf"], n_nb=6)
    assert r["nb_margin"][0] < 1e-6
    # A forced choice evaluates exactly those keyframes (order does not matter).
    nb = r["neighbors"].copy()
    f = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], 1e-3, P["scan"][:8],
                           P["poses"], P["kf"], n_nb=6, neighbors=nb[:, ::-1])
    assert np.allclose(f["loglik"], r["loglik"], rtol=1e-13)
    nb2 = np.tile(np.arange(6, dtype=np.int32), (3, 1))
    f2 = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], 1e-3, P["scan"][:8],
                            P["poses"], P["kf"], n_nb=6, neighbors=nb2)
    assert np.allclose(f2["loglik"], r["loglik"], rtol=1e-13)   # all six either way
    one = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], 1e-3, P["scan"][:8],
                             P["poses"], P["kf"], n_nb=1, neighbors=np.full((3, 1), 3, np.int32))
    Trel = np.linalg.inv(T_of(P["kf"][0, 3])) @ T_of(P["poses"][0])
    ll, _ = oracle.evaluate_f64(P["grids"][3], P["dims"], P["origins"][3], P["h"], 1e-3,
                                P["scan"][:8], pose_of(Trel)[None, :])
    assert abs(one["loglik"][0] - ll[0]) < 1e-9 * abs(ll[0])


def test_sum_over_neighbours_is_additive():
    P = make_problem(2, K=8, N=6)
    eps = 1e-3
    r4 = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], eps, P["scan"], P["poses"],
                            P["kf"], n_nb=4)
    for i in range(6):
        tot_l, tot_g = 0.0, np.zeros(6)
        for k in r4["neighbors"][i]:
            Trel = np.linalg.inv(T_of(P["kf"][i, k])) @ T_of(P["poses"][i])
            ll, g = oracle.evaluate_f64(P["grids"][k], P["dims"], P["origins"][k], P["h"], eps,
                                        P["scan"], pose_of(Trel)[None, :])
            tot_l += ll[0]
            tot_g += g[0]
        assert abs(r4["loglik"][i] - tot_l) < 1e-9 * abs(tot_l)
        assert np.allclose(r4["grad"][i], tot_g, rtol=1e-8, atol=1e-8 * np.abs(tot_g).max())


def test_identity_keyframe_reduces_to_plain_filter():
    P = make_problem(3, K=1, N=5)
    P["kf"][:] = np.array([0, 0, 0, 1, 0, 0, 0], np.float32)
    eps = 1e-3
    r = oracle.kf_evaluate(P["grids"], P["dims"], P["origins"], P["h"], eps, P["scan"], P["poses"],
                           P["kf"], n_nb=1)
    s = oracle.evaluate(P["grids"][0], P["dims"], P["origins"][0], P["h"], eps, P["scan"], P["poses"])
    assert np.allclose(r["loglik"], s["loglik"], rtol=1e-14)
    assert np.allclose(r["grad"], s["grad"], rtol=1e-12, atol=1e-12)
