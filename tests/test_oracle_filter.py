"""Pins of the oracle's whole filter on the linear-Gaussian OU model, where
the optimal filter is the closed-form Kalman filter (CPU only).

Checked against the paper's results:
  - Lemma 2: E[G_t^N] equals the marginal likelihood p(y_{1:t});
  - Theorem 1: the bias of (f, pi_t^N) is O(1/N), resolved and with a log-log
    slope near -1, and it equals the bias of an independent self-normalised
    importance sampler built from numpy's generator with the exact transition;
  - Corollary 2 / Remark 5: at a fixed budget K = MN the ensemble's MSE is
    bias-dominated for N < M and matches the centralised filter for N >= M;
    the ensemble variance is the single-filter variance divided by M;
  - Sec. 3.1: N = 1 means no effective resampling, so the ensemble mean is the
    prior-predictive mean (a closed form here);
  - large K tracks the Kalman mean over many observation times.
"""
import numpy as np
import pytest

import pf_inputs

SPEC_BIAS = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.5)
Y_BIAS = np.array([[2.0]])


def _single_filter_estimates(orc, m, N, y, R, seed0):
    est = np.zeros(R)
    logG = np.zeros(R)
    for r in range(R):
        e, _, lz, _ = orc.run_ensemble(m, seed0 + r, 1, N, y)
        est[r] = e[-1, 0]
        logG[r] = lz[0]
    return est, logG


def _snis_reference(N, R, rng):
    # self-normalised importance sampling with the exact interval transition of
    # the Euler scheme x_S = a x_0 + N(0, q); independent of the oracle.
    phi = 1.0 - 0.01
    a = phi**10
    q = sum(0.01 * phi ** (2 * i) for i in range(10))
    x = a * rng.standard_normal((R, N)) + np.sqrt(q) * rng.standard_normal((R, N))
    lw = -(2.0 - x) ** 2 / (2 * 0.5)
    w = np.exp(lw - lw.max(1, keepdims=True))
    est = (w * x).sum(1) / w.sum(1)
    return est.mean(), est.std() / np.sqrt(R)


def test_bias_order_one_over_n(orc):
    m = orc.Model(SPEC_BIAS)
    kmean, _, _ = orc.kalman_ou(m, Y_BIAS[:, 0])
    rng = np.random.default_rng(12345)
    Ns = [4, 8, 16, 32]
    biases = []
    for N in Ns:
        est, _ = _single_filter_estimates(orc, m, N, Y_BIAS, 6000, 10_000 * N)
        b = est.mean() - kmean[-1]
        se = est.std() / np.sqrt(est.size)
        assert abs(b) > 4 * se, (N, b, se)
        ref, ref_se = _snis_reference(N, 200_000, rng)
        assert abs(est.mean() - ref) < 4 * np.hypot(se, ref_se), (N, est.mean(), ref)
        biases.append(abs(b))
    slope = np.polyfit(np.log(Ns), np.log(biases), 1)[0]
    assert -1.5 <= slope <= -0.5, slope


def test_evidence_unbiased(orc):
    spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 3, 3)
    _, _, ll = orc.kalman_ou(m, y[:, 0])
    _, logG = _single_filter_estimates(orc, m, 8, y, 20000, 500_000)
    ratio = np.exp(logG - ll)
    se = ratio.std() / np.sqrt(ratio.size)
    assert abs(ratio.mean() - 1.0) < 3 * se + 1e-3, (ratio.mean(), se)


def test_mse_budget_split(orc):
    m = orc.Model(SPEC_BIAS)
    kmean, _, _ = orc.kalman_ou(m, Y_BIAS[:, 0])
    K = 256
    R = 300
    mse = {}
    for M in (64, 16, 4, 1):
        N = K // M
        err = np.zeros(R)
        for r in range(R):
            e, _, _, _ = orc.run_ensemble(m, 900_000 + 1000 * M + r, M, N, Y_BIAS)
            err[r] = e[-1, 0] - kmean[-1]
        mse[M] = (err**2).mean()
    # bias-dominated when N < M (Remark 5): N = 4 is far worse than N = 64
    assert mse[64] > 5 * mse[4]
    assert mse[64] > mse[16] > mse[4] * 0.8
    # N >= M: the ensemble matches the centralised filter within sampling error
    assert mse[4] < 1.5 * mse[1] and mse[1] < 1.5 * mse[4]


def test_ensemble_variance_one_over_m(orc):
    m = orc.Model(SPEC_BIAS)
    N = 16
    est, _ = _single_filter_estimates(orc, m, N, Y_BIAS, 4096, 7_000_000)
    v1 = est.var()
    for M in (4, 16):
        grp = np.array([orc.run_ensemble(m, 8_000_000 + M * 10_000 + r, M, N, Y_BIAS)[0][-1, 0]
                        for r in range(512)])
        ratio = grp.var() * M / v1
        # sample-variance ratio with 511 d.o.f.: ~6% relative sd
        assert 0.75 < ratio < 1.3, (M, ratio)


def test_n_equals_one_is_prior_predictive(orc):
    spec = pf_inputs.ou1d(theta=1.0, sd=0.5, h=0.01, S=10, obs_var=0.05, prior_mean=3.0,
                          prior_sd=0.5)
    m = orc.Model(spec)
    T = 5
    _, y = orc.simulate(m, 1, T)
    y = y + 10.0  # observations far away: irrelevant when N = 1
    M = 20000
    est, est_w, _, ess = orc.run_ensemble(m, 4, M, 1, y)
    phi = 1 - 0.01
    a = phi**10
    q = sum(0.5**2 * 0.01 * phi ** (2 * i) for i in range(10))
    var = 0.25
    for t in range(1, T + 1):
        var = a * a * var + q
        assert abs(est[t - 1, 0] - 3.0 * a**t) < 4 * np.sqrt(var / M)
    assert np.allclose(ess, 1.0)
    assert np.allclose(est, est_w)


def test_tracks_kalman_mean(orc):
    spec = pf_inputs.ou1d(theta=0.5, sd=1.0, h=0.01, S=10, obs_var=0.2)
    m = orc.Model(spec)
    T = 30
    _, y = orc.simulate(m, 21, T)
    km, kv, _ = orc.kalman_ou(m, y[:, 0])
    est, est_w, _, _ = orc.run_ensemble(m, 5, 8, 2048, y)
    # K = 16384 particles: squared error ~ Var/K, far below the posterior var
    assert np.mean((est[:, 0] - km) ** 2 / kv) < 0.01
    assert np.mean((est_w[:, 0] - km) ** 2 / kv) < 0.01


def test_ensemble_is_equal_weight_average(orc):
    # Definition 3: (1/M) sum of the M independent filters' estimates
    m = orc.Model(pf_inputs.lorenz63())
    _, y = orc.simulate(m, 2, 4)
    est, _, logZ, _ = orc.run_ensemble(m, 17, 3, 32, y)
    acc = np.zeros_like(est)
    for f in range(3):
        X = orc.init(m, 17, f, 32)
        lz = 0.0
        for t in range(1, 5):
            r = orc.filter_interval(m, 17, f, t, X, y[t - 1], lz)
            X, lz = r["X"], r["logZ"]
            acc[t - 1] += r["mean_post"] / 3
        assert lz == pytest.approx(logZ[f], rel=1e-12)
    assert np.allclose(acc, est, rtol=1e-12, atol=1e-12)


# ---- pins of the prior draw's scale and of the effective sample size ------
# (Algorithm 1 step 1, eq. (eqPrior): x_0 ~ tau_0 = N(mean, diag(sd^2)).)

def _chi2_ratio_ok(s2, var, dof, z=5.0):
    """Sample variance with `dof` degrees of freedom against its law:
    dof s2 / var ~ chi^2(dof), i.e. s2 / var = 1 +- z sqrt(2 / dof)."""
    return abs(s2 / var - 1.0) <= z * np.sqrt(2.0 / dof)


@pytest.mark.parametrize("spec", [
    pf_inputs.ou1d(sd=0.5, prior_mean=3.0, prior_sd=0.5),
    dict(pf_inputs.lorenz63(), prior_sd=[0.5, 2.0, 3.0]),
])
def test_prior_draw_scale(orc, spec):
    """The per-component sample variance of 2e5 prior draws equals prior_sd^2
    within chi-square bounds (a draw scaled by sd^2 or by another component's
    sd fails), the means are the prior means, and the components are
    uncorrelated."""
    m = orc.Model(spec)
    N = 200_000
    X = orc.init(m, 123, 5, N)
    mu = np.asarray(spec["prior_mean"])
    sd = np.asarray(spec["prior_sd"])
    for c in range(m.dx):
        s2 = X[:, c].var(ddof=1)
        assert _chi2_ratio_ok(s2, sd[c] ** 2, N - 1), (c, s2, sd[c] ** 2)
        assert abs(X[:, c].mean() - mu[c]) < 5 * sd[c] / np.sqrt(N)
    if m.dx > 1:
        r = np.corrcoef(X.T)
        assert np.all(np.abs(r[~np.eye(m.dx, dtype=bool)]) < 5 / np.sqrt(N))


def test_prior_draw_scale_fhn_grid(orc):
    """FH-N 4 x 4 grid, prior sd 0.05 on v and w around the stimulus pattern:
    pooled chi-square of the 32 component variances, and the v/w lanes of one
    Philox call independent."""
    spec = pf_inputs.fhn(4)
    m = orc.Model(spec)
    N = 20_000
    X = orc.init(m, 7, 1, N)
    mu = np.asarray(spec["prior_mean"])
    dev = (X - mu) / 0.05
    pooled = (dev ** 2).sum() / (N * m.dx)
    assert _chi2_ratio_ok(pooled, 1.0, N * m.dx)
    assert np.all(np.abs(dev.mean(0)) < 5 / np.sqrt(N))
    # v and w of node 0 come from lanes 0 and 1 of the same call
    assert abs(np.corrcoef(X[:, 0], X[:, 16])[0, 1]) < 5 / np.sqrt(N)


def test_prior_predictive_variance_ou(orc):
    """N particles of one filter propagated without resampling from the
    prior: after t intervals the sample variance is the closed form
    a^2 var + q of the discrete OU recursion (pins the prior's scale together
    with the Euler noise)."""
    spec = pf_inputs.ou1d(theta=1.0, sd=0.5, h=0.01, S=10, prior_mean=3.0, prior_sd=0.5)
    m = orc.Model(spec)
    N = 200_000
    X = orc.init(m, 9, 0, N)
    phi = 1 - 0.01
    a = phi ** 10
    q = sum(0.5 ** 2 * 0.01 * phi ** (2 * i) for i in range(10))
    var, mean = 0.25, 3.0
    for t in range(1, 4):
        X = orc.propagate(m, 9, 0, t, X)
        var = a * a * var + q
        mean = a * mean
        assert _chi2_ratio_ok(X[:, 0].var(ddof=1), var, N - 1), (t, X[:, 0].var(), var)
        assert abs(X[:, 0].mean() - mean) < 5 * np.sqrt(var / N)


def test_ess_hand_values(orc):
    """ESS = (sum w)^2 / sum w^2 on hand-computed weight vectors with N > 1."""
    with np.errstate(divide="ignore"):
        assert orc.ess(np.log([1.0, 1.0, 0.0, 0.0])) == pytest.approx(2.0, rel=1e-15)
    assert orc.ess(np.log([1.0, 2.0, 3.0])) == pytest.approx(36.0 / 14.0, rel=1e-14)
    assert orc.ess(np.zeros(7)) == pytest.approx(7.0, rel=1e-15)
    assert orc.ess(np.array([0.0, -800.0, -900.0])) == pytest.approx(1.0, rel=1e-15)
    # invariant to a common shift of the log-weights
    lw = np.log([0.5, 0.25, 0.125, 0.125])
    e = orc.ess(lw)
    assert e == pytest.approx(1.0 / (0.25 + 0.0625 + 2 * 0.015625), rel=1e-14)
    assert orc.ess(lw - 1000.0) == pytest.approx(e, rel=1e-14)
    # no positive weight: uniform, ESS = N
    assert orc.ess(np.full(5, -np.inf)) == pytest.approx(5.0)


def test_filter_interval_reports_the_ess_of_its_weights(orc):
    m = orc.Model(pf_inputs.lorenz63())
    _, y = orc.simulate(m, 4, 1)
    X = orc.init(m, 3, 0, 64)
    r = orc.filter_interval(m, 3, 0, 1, X, y[0])
    assert 1.0 < r["ess"] < 64.0
    assert r["ess"] == pytest.approx(orc.ess(r["lw"]), rel=1e-14)
