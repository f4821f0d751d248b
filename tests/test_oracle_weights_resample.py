"""Pins for importance weighting (Eq. 11), normalisation and systematic resampling.

References: extended-precision (80-bit) log-sum-exp, exact rational arithmetic
on dyadic weights, and the counting invariants of systematic resampling.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def lse_longdouble(x):
    x = np.asarray(x, np.longdouble)
    m = x.max()
    return m + np.log(np.sum(np.exp(x - m)))


@pytest.mark.parametrize("N", [1, 2, 7, 100, 4096])
def test_logsumexp_and_normalisation(N):
    rng = np.random.default_rng(N)
    logw = rng.normal(size=N) * 30 - 1000
    ll = rng.normal(size=N) * 50
    out, L, ess = oracle.weights(logw, ll, beta=1.0)
    ref = lse_longdouble(logw + ll)
    assert abs(L - float(ref)) <= 4e-16 * abs(float(ref)) + 1e-13
    # logw - L carries an absolute rounding of about ulp(|L|), so sum(w) is 1 to
    # within a few |L| * 2^-52.
    assert abs(math.fsum(np.exp(out)) - 1.0) < 4 * 2.0 ** -52 * (abs(L) + 1.0)
    w = np.exp(np.asarray(out, np.longdouble))
    assert ess == pytest.approx(float(1.0 / np.sum(w * w)), rel=1e-13)


def test_weights_invariances():
    rng = np.random.default_rng(1)
    N = 500
    logw = rng.normal(size=N)
    a, La, Ea = oracle.weights(logw, None)
    b, Lb, Eb = oracle.weights(logw + 12345.0, None)
    assert np.allclose(a, b, atol=1e-9)
    assert Eb == pytest.approx(Ea, rel=1e-10)
    u, _, Eu = oracle.weights(np.full(N, 3.0), None)
    assert Eu == pytest.approx(N, rel=1e-13)
    one = np.full(N, -np.inf)
    one[17] = -5.0
    o, Lo, Eo = oracle.weights(one, None)
    assert Eo == 1.0 and Lo == -5.0 and o[17] == 0.0
    beta_half, _, _ = oracle.weights(np.zeros(N), rng.normal(size=N), beta=0.0)
    assert np.allclose(beta_half, -math.log(N), atol=1e-14)


def systematic_exact(w_frac, u_frac):
    N = len(w_frac)
    cdf, s = [], Fraction(0)
    for w in w_frac:
        s += w
        cdf.append(s)
    out = []
    for k in range(N):
        uk = (u_frac + k) / N
        a = next((i for i in range(N) if cdf[i] > uk), N - 1)
        out.append(a)
    return out


def test_brute_force_dyadic_weights():
    rng = np.random.default_rng(2)
    for trial in range(300):
        N = int(rng.integers(1, 9))
        parts = rng.integers(0, 9, N)
        if parts.sum() == 0:
            parts[0] = 1
        # Dyadic weights summing to one: k/2^m.
        tot = int(parts.sum())
        m = 1 << int(math.ceil(math.log2(tot)))
        parts = parts.copy()
        parts[0] += m - tot
        w = [Fraction(int(p), m) for p in parts]
        u = Fraction(int(rng.integers(0, 1 << 20)) * 2 + 1, 1 << 21)   # never lands on a tie
        logw = np.array([math.log(float(x)) if x > 0 else -np.inf for x in w])
        a, margin = oracle.resample(logw, float(u))
        assert list(a) == systematic_exact(w, u), (trial, w, u)


def test_counting_invariants():
    rng = np.random.default_rng(3)
    for N in (1, 5, 64, 1000, 20000):
        logw = rng.normal(size=N) * 2
        lw, _, _ = oracle.weights(logw, None)
        u = float(rng.uniform())
        a, margin = oracle.resample(lw, u)
        assert a.shape == (N,) and a.min() >= 0 and a.max() < N
        assert np.all(np.diff(a) >= 0)
        counts = np.bincount(a, minlength=N)
        assert counts.sum() == N
        Nw = N * np.exp(lw)
        assert np.all(counts >= np.floor(Nw - 1e-9)) and np.all(counts <= np.ceil(Nw + 1e-9))
        # The margin is the distance from u_k to the nearest CDF value.
        cdf = np.cumsum(np.exp(lw))
        uk = (u + np.arange(N)) / N
        ref = np.abs(cdf[None, :] - uk[:, None]).min(axis=1) if N <= 1000 else None
        if ref is not None:
            assert np.allclose(margin, ref, rtol=0, atol=1e-15)


def test_special_cases():
    N = 1000
    a, _ = oracle.resample(np.full(N, -math.log(N)), 0.5)
    assert np.array_equal(a, np.arange(N))
    lw = np.full(N, -np.inf)
    lw[123] = 0.0
    a, _ = oracle.resample(lw, 0.999)
    assert np.all(a == 123)


def test_unbiased_over_offsets():
    rng = np.random.default_rng(4)
    N = 16
    lw, _, _ = oracle.weights(rng.normal(size=N), None)
    w = np.exp(lw)
    tot = np.zeros(N)
    R = 10000
    for u in rng.uniform(size=R):
        a, _ = oracle.resample(lw, float(u))
        tot += np.bincount(a, minlength=N)
    mean = tot / R
    # Each count takes floor(Nw) or floor(Nw)+1, so its sd is at most 1/2.
    assert np.all(np.abs(mean - N * w) < 4 * 0.5 / math.sqrt(R))


def test_exact_ties_use_strict_inequality():
    """a_k = min{i : CDF_i > u_k}: a u_k that equals a CDF value goes to the next particle."""
    for N in (2, 4):
        w = 1.0 / N
        lw = np.full(N, math.log(w))
        assert math.exp(lw[0]) == w          # the tie is exact in FP64 for these N
        a, margin = oracle.resample(lw, 0.0)  # u_k = k/N = CDF_{k-1} exactly
        assert np.array_equal(a, np.arange(N))
        assert margin[1:].max() == 0.0
        assert list(a) == systematic_exact([Fraction(1, N)] * N, Fraction(0))
    # A zero-weight particle in front: CDF_0 = 0 = u_0 must not select it.
    lw = np.array([-np.inf, 0.0, -np.inf, -np.inf])
    a, _ = oracle.resample(lw, 0.0)
    assert list(a) == [1, 1, 1, 1]
