"""Helpers for the GPU-vs-oracle parity tests (stage-wise protocol).

Tolerances (stated per result):
* log-likelihood: |l_gpu - l_ref| <= 1e-5 |l_ref| + amb_l
* gradient:       |g_gpu,c - g_ref,c| <= 1e-4 sum_j |dl_j/dxi_c| + amb_g,c
  where amb_* is the oracle's allowance for points whose index coordinate is
  within DELTA of a cell face, where the two sides' cell choices could differ
  and the interpolant's one-sided derivative with it.  The kernel forms u in
  FP64 from the same FP32 inputs, so the two agree on u to about 1e-12 index
  units and DELTA = 1e-9 covers that; such points are counted (none is
  expected) and the reported errors are taken over every particle.
* pose step (oracle fed the GPU's own gradient): translation within 4 FP32
  ulps of |t| plus 1e-7 m, rotation within 2e-6 rad.
* log-sum-exp: relative 1e-13; ESS: relative 1e-10.
* resampled indices: bit-exact except where the oracle's CDF is within 1e-12
  of u_k (counted).
* neighbour keyframes: bit-exact except for particles whose FP64 ranking has
  two consecutive squared distances (of distinct translations) within a
  relative NB_TIE of each other (counted); there the kernel's FP32 ranking may
  order them either way, so its choice is checked to be a valid nearest set
  and the likelihood is compared with the oracle evaluated on that choice.
"""

import math

import numpy as np

import oracle

DELTA = 1e-9          # index units; bound on |u_kernel - u_oracle| (both FP64 transforms)
TIE = 1e-12
# An FP32 squared distance ((dx^2 + dy^2) + dz^2), dx rounded from the FP32
# translations, carries at most about 5 rounding errors of 2^-24 relative to
# the exact value (every term is non-negative); two such errors apart is below
# 6e-7, so a relative gap of 1e-6 cannot be reordered.
NB_TIE = 1e-6


def quat_angle(qa, qb):
    """Rotation angle between unit quaternions (rows), sign-invariant."""
    qa = np.asarray(qa, np.float64)
    qb = np.asarray(qb, np.float64)
    qa = qa / np.linalg.norm(qa, axis=-1, keepdims=True)
    qb = qb / np.linalg.norm(qb, axis=-1, keepdims=True)
    d = np.abs(np.sum(qa * qb, axis=-1)).clip(0, 1)
    return 2.0 * np.arccos(d)


def ulp32(x):
    x = np.abs(np.asarray(x, np.float32))
    return np.spacing(x).astype(np.float64)


def check_eval(loglik, grad, ref, idx=None, report=None):
    """Compare GPU l, g (rows idx of the oracle's arrays) with the oracle."""
    if idx is None:
        idx = np.arange(len(loglik))
    l_ref, g_ref = ref["loglik"][idx], ref["grad"][idx]
    dl = np.abs(loglik.astype(np.float64) - l_ref)
    tol_l = 1e-5 * np.abs(l_ref) + ref["amb_l"][idx]
    dg = np.abs(grad.astype(np.float64) - g_ref)
    tol_g = 1e-4 * ref["gabs"][idx] + ref["amb_g"][idx] + 1e-6
    bad_l = np.nonzero(dl > tol_l)[0]
    bad_g = np.nonzero(np.any(dg > tol_g, axis=1))[0]
    if report is not None:
        rel_l = dl / np.maximum(np.abs(l_ref), 1e-30)
        rel_g = dg / np.maximum(ref["gabs"][idx], 1e-30)
        report.update(max_rel_l=float(rel_l.max()), max_rel_g=float(rel_g.max()),
                      n_amb=int(ref["n_amb"][idx].sum()), n=len(idx))
    assert bad_l.size == 0, "loglik off for %d particles, first %d: %r vs %r (tol %r)" % (
        bad_l.size, idx[bad_l[0]], loglik[bad_l[0]], l_ref[bad_l[0]], tol_l[bad_l[0]])
    if bad_g.size:
        rel = dg / np.maximum(ref["gabs"][idx], 1e-30)
        w = int(np.argmax(rel.max(axis=1)))
        raise AssertionError("grad off for %d particles, first %d: %r vs %r; worst %d: rel %r "
                             "(scale %r)" % (bad_g.size, idx[bad_g[0]], grad[bad_g[0]],
                                             g_ref[bad_g[0]], idx[w], rel[w], ref["gabs"][idx][w]))


def check_step(poses_in, grad_gpu, poses_gpu, params):
    """Oracle step from the GPU's gradient vs the GPU's stepped poses (rows aligned)."""
    ref = oracle.step(poses_in, grad_gpu.astype(np.float64), params["alpha_t"], params["alpha_r"],
                      params["rho_max"], params["phi_max"])
    dt = np.abs(poses_gpu[:, :3].astype(np.float64) - ref[:, :3])
    tol_t = 4 * ulp32(ref[:, :3]) + 1e-7
    assert np.all(dt <= tol_t), "translation off by %g (tol %g)" % (dt.max(), tol_t.max())
    ang = quat_angle(poses_gpu[:, 3:], ref[:, 3:])
    assert np.all(ang <= 2e-6), "rotation off by %g rad" % ang.max()
    return ref


def check_weights_resample(logw_in, loglik_gpu, beta, u, out, policy, ess_frac=0.5):
    """Weights and resampling, the oracle fed the GPU's likelihoods."""
    N = len(logw_in)
    beta = float(np.float32(beta))       # the step parameters carry beta in FP32
    lw_ref, L, ess = oracle.weights(logw_in, loglik_gpu.astype(np.float64), beta)
    st = out["stats"]
    assert abs(st["lse"] - L) <= 1e-13 * max(1.0, abs(L)), (st["lse"], L)
    assert abs(st["ess"] - ess) <= 1e-10 * ess, (st["ess"], ess)
    pre = np.asarray(logw_in, np.float64) + beta * loglik_gpu.astype(np.float64)
    best = int(np.argmax(pre))
    assert st["best"] == best
    fire = {0: False, 1: True, 2: ess < ess_frac * N}[policy]
    near_trigger = policy == 2 and abs(ess - ess_frac * N) < 1e-9 * N
    if not near_trigger:
        assert st["resampled"] == fire
    n_tie = 0
    if st["resampled"]:
        a_ref, margin = oracle.resample(lw_ref, u)
        mism = np.nonzero(out["parents"] != a_ref)[0]
        n_tie = int(np.sum(margin < TIE))
        assert np.all(margin[mism] < TIE), "resampled index mismatch at k=%d (%d vs %d)" % (
            mism[0], out["parents"][mism[0]], a_ref[mism[0]])
        assert np.allclose(out["logw"], -math.log(N), rtol=0, atol=1e-15)
    else:
        assert np.array_equal(out["parents"], np.arange(N))
        assert np.allclose(out["logw"], lw_ref, rtol=0, atol=1e-13 * max(1.0, abs(L)))
    return dict(lse=L, ess=ess, ties=n_tie)


def check_loop_update(poses_in, kf_in, out, params, n_recent):
    """Loop-gated correction (Eq. 5-10), the oracle fed the GPU's gradient and
    neighbours: loop flags exact; untouched poses bit-exact; moved poses within
    the step tolerances.  Returns the oracle's result."""
    ref = oracle.kf_loop_update(poses_in, kf_in, out["grad"].astype(np.float64), out["neighbors"],
                                params, n_recent=n_recent)
    loop = ref["loop"] >= 0
    P, KP = out["poses"], out["kf_poses"]
    # Not corrected: the translation is untouched, the quaternion only renormalised.
    assert np.array_equal(P[~loop, :3], poses_in[~loop, :3]), "a particle without a loop moved"
    assert np.all(quat_angle(P[~loop, 3:], poses_in[~loop, 3:]) <= 1e-6)
    assert np.array_equal(KP[~loop], kf_in[~loop]), "keyframes of a particle without a loop moved"
    N, K = KP.shape[:2]
    o = np.where(loop, ref["loop"], K)
    before = np.arange(K)[None, :] <= o[:, None]
    assert np.array_equal(KP[before], kf_in[before]), "a keyframe at or before the oldest neighbour moved"
    for got, want in ((P[loop], ref["poses"][loop]), (KP[loop].reshape(-1, 7), ref["kf_poses"][loop].reshape(-1, 7))):
        dt = np.abs(got[:, :3].astype(np.float64) - want[:, :3])
        tol = 4 * ulp32(want[:, :3]) + 2e-7
        assert np.all(dt <= tol), "translation off by %g (tol %g)" % (dt.max(), tol.max())
        ang = quat_angle(got[:, 3:], want[:, 3:])
        assert np.all(ang <= 2e-6), "rotation off by %g rad" % ang.max()
    return ref


def check_prune(logw_in, loglik_gpu, beta, u, out, tau_post, tau_lik):
    """Dead-particle pruning (Sec. III-F), the oracle fed the GPU's likelihoods:
    dead count and parents exact except near-ties of the systematic draw,
    log-weights to rounding, respawned poses bit-exact copies of the parent's.
    Returns the oracle's result."""
    beta = float(np.float32(beta))
    tau_post, tau_lik = float(np.float32(tau_post)), float(np.float32(tau_lik))
    l64 = loglik_gpu.astype(np.float64)
    lw_ref, L, ess = oracle.weights(logw_in, l64, beta)
    r = oracle.prune(lw_ref, l64, tau_post, tau_lik, u)
    # A dead decision taken within rounding of the threshold is not checked.
    assert not np.any(np.abs(lw_ref - np.log(tau_post)) < 1e-9), "near-tie in the weight test"
    st = out["stats"]
    assert st["pruned"] == r["n_dead"], (st["pruned"], r["n_dead"])
    par = out["parents"]
    ties = r["margin"] < 1e-12
    mism = par != r["parents"]
    assert np.all(ties[mism]), "parents differ away from ties: %s" % np.flatnonzero(mism & ~ties)[:10]
    ok = ~mism
    dl = np.abs(out["logw"][ok] - r["logw"][ok])
    fin = np.isfinite(r["logw"][ok])
    assert np.all(dl[fin] <= 1e-12 + 1e-12 * np.abs(r["logw"][ok][fin])), dl[fin].max()
    dead = par != np.arange(len(par))
    assert np.array_equal(out["poses"][dead], out["poses"][par[dead]])
    assert abs(np.sum(np.exp(out["logw"])) - 1.0) < 1e-10
    return r


def check_neighbors(nb_gpu, ref, poses, kf_poses):
    """Neighbour choice: bit-exact away from counted near-ties, else a valid
    nearest set (each chosen keyframe within NB_TIE of the n-th FP64 distance).
    Returns the boolean mask of particles whose choice differs from the oracle's."""
    nb_gpu = np.asarray(nb_gpu)
    tie = ref["nb_margin"] < NB_TIE
    diff = np.any(nb_gpu != ref["neighbors"], axis=1)
    assert not np.any(diff & ~tie), "neighbours differ away from near-ties at %s" % (
        np.flatnonzero(diff & ~tie)[:10])
    n = nb_gpu.shape[1]
    for i in np.flatnonzero(diff):
        t = np.asarray(poses[i, :3], np.float64)
        d2 = np.sum((np.asarray(kf_poses[i, :, :3], np.float64) - t) ** 2, axis=1)
        lim = np.sort(d2)[n - 1] * (1 + NB_TIE)
        assert len(set(nb_gpu[i].tolist())) == n and np.all(d2[nb_gpu[i]] <= lim), i
    return diff
