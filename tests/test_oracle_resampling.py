"""Pins of the oracle's weighting, normalisation and multinomial resampling
(Algorithm 1, steps 2(a)-2(b)); CPU only.

Pins: scipy's Beta and uniform distributions for the sorted uniforms, numpy's
searchsorted for the ancestor search, chi-square tests against the exact
multinomial law (scipy) for the offspring counts.
"""
import itertools

import numpy as np
import pytest
from scipy import stats


def test_sorted_uniforms_are_order_statistics(orc):
    N = 16
    R = 4000
    U = np.array([orc.sorted_uniforms(5, 1, t, N) for t in range(1, R + 1)])
    assert np.all(np.diff(U, axis=1) >= 0)
    assert np.all((U > 0) & (U < 1))
    # k-th order statistic of N uniforms ~ Beta(k+1, N-k)
    for k in (0, 5, N - 1):
        assert stats.kstest(U[:, k], stats.beta(k + 1, N - k).cdf).pvalue > 1e-4
    # the unordered values are uniform
    assert stats.kstest(U.ravel()[:: 3], "uniform").pvalue > 1e-4


def test_sorted_uniforms_first_is_beta_large_n(orc):
    N = 1000
    U0 = np.array([orc.sorted_uniforms(9, 0, t, N)[0] for t in range(1, 3001)])
    assert stats.kstest(U0, stats.beta(1, N).cdf).pvalue > 1e-4


def test_ancestors_match_searchsorted(orc):
    rng = np.random.default_rng(2)
    for N in (1, 2, 7, 64, 1000):
        w = rng.random(N) ** 3
        w[rng.random(N) < 0.2] = 0.0
        w[-1] += 1e-3
        C = np.cumsum(w)
        U = np.sort(rng.random(N))
        A = orc.ancestors(C, U)
        ref = np.searchsorted(C, U * C[-1], side="right")
        assert np.array_equal(A, np.minimum(ref, N - 1))
        # zero-weight particles are never selected
        assert np.all(w[A] > 0)


def test_ancestor_tie_goes_to_next(orc):
    C = np.array([1.0, 2.0, 3.0, 4.0])
    U = np.array([0.25, 0.5, 0.5, 0.75])
    # U*C_N = 1, 2, 2, 3 lie exactly on C_0, C_1, C_1, C_2: strict '>' picks i+1
    assert list(orc.ancestors(C, U)) == [1, 2, 2, 3]


def test_normalise_shift_invariance_and_degenerate(orc):
    lw = np.array([-3.0, -1.0, -2.0, -7.5])
    mx, W, s2, deg = orc.normalise(lw)
    assert mx == -1.0 and not deg
    mx2, W2, s22, _ = orc.normalise(lw + 123.0)
    assert W2 == pytest.approx(W, rel=1e-15) and mx2 == mx + 123.0
    assert W == pytest.approx(np.exp(-2) + 1 + np.exp(-1) + np.exp(-6.5), rel=1e-15)
    mx, W, s2, deg = orc.normalise(np.full(5, -np.inf))
    assert deg and W == 5.0
    C = orc.cdf(np.full(5, -np.inf), mx, deg)
    assert list(C) == [1, 2, 3, 4, 5]


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_multinomial_marginal_counts_chi2(orc, N):
    rng = np.random.default_rng(N)
    w = rng.random(N) + 0.05
    w /= w.sum()
    lw = np.log(w)
    R = 12000
    counts = np.zeros(N)
    for t in range(1, R + 1):
        A, *_ = orc.resample(77, 3, t, lw)
        counts += np.bincount(A, minlength=N)
    expected = R * N * w
    chi2, p = stats.chisquare(counts, expected)
    assert p > 1e-4


def test_multinomial_joint_law_n3(orc):
    w = np.array([0.2, 0.5, 0.3])
    lw = np.log(w)
    R = 20000
    comps = [c for c in itertools.product(range(4), repeat=3) if sum(c) == 3]
    index = {c: i for i, c in enumerate(comps)}
    obs = np.zeros(len(comps))
    for t in range(1, R + 1):
        A, *_ = orc.resample(11, 0, t, lw)
        obs[index[tuple(np.bincount(A, minlength=3))]] += 1
    pmf = np.array([stats.multinomial.pmf(c, 3, w) for c in comps])
    chi2, p = stats.chisquare(obs, R * pmf)
    assert p > 1e-4
