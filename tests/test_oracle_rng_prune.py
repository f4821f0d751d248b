"""Pins for the oracle's prediction-noise generator and dead-particle pruning.

Generator: SplitMix64's published reference outputs for seed 0, a
Kolmogorov-Smirnov test of the Box-Muller normals against scipy's normal CDF,
moments and pair correlations, and the counter property (a particle's
numbers do not depend on how many particles are drawn).

Pruning (Sec. III-F): the definition evaluated with exact rational arithmetic
on dyadic weights (brute force on tiny inputs), plus invariants that hold at
any size: weights sum to one, live particles keep their state, every copy
has a live parent, copy counts are the floor or ceiling of D w_p / W, and a
parent's weight is shared equally with its copies.
"""

from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle


def test_splitmix64_reference_outputs():
    # First outputs of SplitMix64 seeded with 0 (Steele, Lea and Flood's generator).
    got = [int(x) for x in oracle.splitmix64(0, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_normals_are_standard_normal():
    z = oracle.rng_normals(12345, 7, 100000)
    for c in range(6):
        ks = stats.kstest(z[:, c], "norm")
        assert ks.pvalue > 1e-3, (c, ks)
        assert abs(z[:, c].mean()) < 0.02 and abs(z[:, c].std() - 1.0) < 0.02
    corr = np.corrcoef(z.T)
    assert np.max(np.abs(corr - np.eye(6))) < 0.02


def test_normals_are_counter_based():
    a = oracle.rng_normals(99, 3, 10)
    b = oracle.rng_normals(99, 3, 1000)
    assert np.array_equal(a, b[:10])
    c = oracle.rng_normals(99, 4, 10)
    d = oracle.rng_normals(98, 3, 10)
    assert not np.any(a == c) and not np.any(a == d)


def test_predict_rng_applies_scaled_normals():
    rng = np.random.default_rng(3)
    poses = np.concatenate([rng.normal(size=(20, 3)), rng.normal(size=(20, 4))], axis=1).astype(np.float32)
    dT = np.array([0.3, -0.1, 0.05, 0.99, 0.05, -0.08, 0.02])
    dT[3:] /= np.linalg.norm(dT[3:])
    sigma = np.array([0.05, 0.05, 0.02, 0.01, 0.01, 0.03])
    want = oracle.predict(poses, dT, (sigma * oracle.rng_normals(5, 11, 20)).astype(np.float32))
    got = oracle.predict_rng(poses, dT, 5, 11, sigma)
    # The oracle's plain prediction takes FP32 noise; the generated one is FP64.
    assert np.allclose(got, want, atol=2e-7)


def exact_prune(w, lik, tau_post, tau_lik, u):
    """The pruning definition in exact rational arithmetic (w: Fractions summing to 1)."""
    N = len(w)
    lmax = max(lik)
    dead = [bool(w[i] < tau_post or lik[i] - lmax < np.log(tau_lik)) for i in range(N)]
    D = sum(dead)
    live = [i for i in range(N) if not dead[i]]
    par = list(range(N))
    new = list(w)
    if D == 0 or not live:
        return par, new, 0
    W = sum(w[i] for i in live)
    cdf, c = [], Fraction(0)
    for i in range(N):
        if not dead[i]:
            c += w[i]
        cdf.append(c)
    copies = [0] * N
    k = 0
    for s in range(N):
        if not dead[s]:
            continue
        target = (Fraction(u) + k) / D * W
        a = next((i for i in range(N) if cdf[i] > target), live[-1])
        par[s] = a
        copies[a] += 1
        k += 1
    for p in live:
        new[p] = w[p] / (1 + copies[p]) / W
    for s in range(N):
        if dead[s]:
            new[s] = new[par[s]]
    return par, new, D


@pytest.mark.parametrize("seed", range(12))
def test_prune_matches_exact_definition_on_dyadic_weights(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 9))
    num = rng.integers(0, 9, N)
    num[rng.integers(N)] += 1                       # at least one positive weight
    w = [Fraction(int(x), int(num.sum())) for x in num]
    # Dyadic weights: round to multiples of 1/64 keeping the sum exact.
    q = [Fraction(int(round(float(x) * 64)), 64) for x in w]
    q[int(np.argmax(num))] += 1 - sum(q)
    if any(x < 0 for x in q):
        pytest.skip("rounding made a negative weight")
    lik = rng.normal(size=N) * 10
    u = float(Fraction(int(rng.integers(0, 64)), 64))
    tau_post = 1.0 / 32
    tau_lik = float(np.exp(-12.0))
    logw = np.array([np.log(float(x)) if x > 0 else -np.inf for x in q])
    par, new, D = exact_prune(q, lik, tau_post, tau_lik, u)
    r = oracle.prune(logw, lik, tau_post, tau_lik, u)
    assert r["n_dead"] == D
    assert list(r["parents"]) == par
    want = np.array([np.log(float(x)) if x > 0 else -np.inf for x in new])
    fin = np.isfinite(want)
    assert np.array_equal(np.isfinite(r["logw"]), fin)
    assert np.allclose(r["logw"][fin], want[fin], rtol=0, atol=1e-14)


def test_prune_invariants_at_size():
    rng = np.random.default_rng(21)
    N = 5000
    logw = rng.normal(size=N) * 6
    logw -= np.log(np.sum(np.exp(logw)))
    lik = rng.normal(size=N) * 20
    tau_post, tau_lik = 1e-8, 1e-16
    r = oracle.prune(logw, lik, tau_post, tau_lik, 0.37)
    dead = (logw < np.log(tau_post)) | (lik - lik.max() < np.log(tau_lik))
    D = int(dead.sum())
    assert r["n_dead"] == D > 100
    par = r["parents"]
    assert np.array_equal(par[~dead], np.flatnonzero(~dead))
    assert not np.any(dead[par[dead]])
    w = np.exp(logw)
    W = w[~dead].sum()
    copies = np.bincount(par[dead], minlength=N)
    expect = D * w / W
    live = ~dead
    assert np.all(copies[live] >= np.floor(expect[live] - 1e-9))
    assert np.all(copies[live] <= np.ceil(expect[live] + 1e-9))
    assert abs(np.sum(np.exp(r["logw"])) - 1.0) < 1e-12
    assert np.allclose(r["logw"][dead], r["logw"][par[dead]], rtol=0, atol=0)
    # Each parent's weight is split equally with its copies.
    assert np.allclose(np.exp(r["logw"][live]) * (1 + copies[live]), w[live] / W, rtol=1e-12)


def test_prune_likelihood_criterion_and_no_dead():
    logw = np.log(np.array([0.4, 0.3, 0.2, 0.1]))
    lik = np.array([-10.0, -10.0 - 40.0, -11.0, -9.0])     # particle 1: likelihood ratio e^-40
    r = oracle.prune(logw, lik, 1e-8, 1e-16, 0.5)
    assert r["n_dead"] == 1 and r["parents"][1] != 1
    r0 = oracle.prune(logw, np.array([-10.0, -10.5, -11.0, -9.0]), 1e-8, 1e-16, 0.5)
    assert r0["n_dead"] == 0
    assert np.array_equal(r0["parents"], np.arange(4)) and np.array_equal(r0["logw"], logw)
