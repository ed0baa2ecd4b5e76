"""Pins of the oracle's other resampling schemes and of the ESS-triggered
schedule (Sec. 2.3: the convergence results hold for other schemes than
multinomial); CPU only.

Pins from the schemes' definitions and known laws, not from the oracle's
own formulas:
  - every scheme is unbiased, E[n_i] = N w_i / W (offspring counts n_i);
  - systematic: n_i is floor or ceil of N w_i / W, and the ceiling occurs
    with probability equal to the fractional part (one uniform offset over
    a lattice of spacing 1/N);
  - stratified: one point per stratum, so a particle whose weight covers
    whole strata is always chosen for them;
  - residual: n_i >= floor(N w_i / W) always, and the remaining draws follow
    the multinomial law of the fractional parts (chi-square against scipy);
  - ascending ancestors, N in total, zero-weight particles never chosen;
  - the schedule at threshold 0 is Algorithm 1 (or_filter_interval) exactly;
    never resampling is sequential importance sampling, checked against an
    independent numpy accumulation of the path log-weights; on the OU model
    the ESS-scheduled filter keeps E[G] = p(y) (Lemma 2) and tracks the
    closed-form Kalman mean.
"""
import numpy as np
import pytest
from scipy import stats

import pf_inputs

SCHEMES = ("multinomial", "systematic", "stratified", "residual")


def _counts(A, N):
    return np.bincount(A, minlength=N)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_schemes_are_unbiased(orc, scheme):
    w = np.array([0.05, 0.3, 0.0, 0.15, 0.5])
    N = w.size
    lw = np.log(np.where(w > 0, w, 1e-300))
    lw[w == 0] = -np.inf
    R = 20000
    cnt = np.array([_counts(orc.resample_scheme(scheme, 3, 0, t, lw), N) for t in range(1, R + 1)])
    assert np.all(cnt.sum(1) == N)
    assert np.all(cnt[:, 2] == 0)
    mean = cnt.mean(0)
    se = cnt.std(0) / np.sqrt(R) + 1e-12
    assert np.all(np.abs(mean - N * w) <= 5 * se + 1e-9), (mean, N * w, se)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_ancestors_ascending_and_valid(orc, scheme):
    rng = np.random.default_rng(4)
    for N in (1, 2, 3, 17, 256, 1000):
        lw = np.log(rng.random(N) ** 3 + 1e-6)
        lw[rng.random(N) < 0.2] = -np.inf
        lw[0] = 0.0
        A = orc.resample_scheme(scheme, 9, 2, 5, lw)
        assert A.size == N and np.all(np.diff(A) >= 0)
        assert np.all(np.isfinite(lw[A]))


def test_systematic_counts_are_floor_or_ceil(orc):
    rng = np.random.default_rng(5)
    N = 12
    w = rng.random(N)
    nw = N * w / w.sum()
    lw = np.log(w)
    R = 20000
    cnt = np.array([_counts(orc.resample_scheme("systematic", 8, 1, t, lw), N)
                    for t in range(1, R + 1)])
    lo, hi = np.floor(nw), np.ceil(nw)
    assert np.all((cnt == lo) | (cnt == hi))
    # P(n_i = ceil) = frac(N w_i / W)
    frac = nw - lo
    p = (cnt == hi).mean(0)
    se = np.sqrt(frac * (1 - frac) / R) + 1e-12
    assert np.all(np.abs(p - frac) <= 5 * se), (p, frac)


def test_systematic_uniforms_lattice(orc):
    U = orc.systematic_uniforms(2, 0, 7, 10)
    d = np.diff(U)
    assert np.allclose(d, 0.1, atol=1e-15)
    assert 0 < U[0] < 0.1


def test_stratified_one_point_per_stratum(orc):
    N = 50
    for t in range(1, 40):
        U = orc.stratified_uniforms(2, 1, t, N)
        assert np.all(np.floor(U * N) == np.arange(N))
    # the within-stratum offsets are uniform and independent of the stratum
    off = np.concatenate([orc.stratified_uniforms(6, 0, t, N) * N - np.arange(N)
                          for t in range(1, 201)])
    assert stats.kstest(off, "uniform").pvalue > 1e-4
    # a particle holding whole strata is chosen for each of them
    w = np.array([1.0, 2.0, 1.0])
    A = orc.resample_scheme("stratified", 1, 0, 1, np.log(w))
    c = _counts(A, 3)
    assert c[1] >= 1


def test_residual_deterministic_part_and_residual_law(orc):
    w = np.array([0.1, 0.23, 0.37, 0.3])
    N = 7
    # N = 7 particles: repeat the pattern so that N w_i / W has integer parts
    lw = np.log(np.array([w[i % 4] for i in range(N)]))
    ww = np.exp(lw) / np.exp(lw).sum()
    nw = N * ww
    fl = np.floor(nw)
    R = int(N - fl.sum())
    r = (nw - fl) / (nw - fl).sum()
    reps = 20000
    extra = np.zeros(N)
    for t in range(1, reps + 1):
        c = _counts(orc.resample_scheme("residual", 4, 3, t, lw), N)
        assert np.all(c >= fl)
        extra += c - fl
    exp = reps * R * r
    chi2 = ((extra - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, N - 1) > 1e-4, (extra, exp)


def test_residual_integer_weights_are_deterministic(orc):
    # N = 4, N w / W = (1, 1, 2, 0): no residual draws, the copies in index
    # order whatever the random numbers
    lw4 = np.log(np.array([0.25, 0.25, 0.5, 1.0]))
    lw4[3] = -np.inf
    for t in range(1, 20):
        assert list(orc.resample_scheme("residual", 1, 0, t, lw4)) == [0, 1, 2, 2]


@pytest.mark.parametrize("scheme", SCHEMES)
def test_degenerate_weights_resample_uniformly(orc, scheme):
    N = 8
    lw = np.full(N, -np.inf)
    A = orc.resample_scheme(scheme, 1, 0, 3, lw)
    assert A.size == N and np.all(np.diff(A) >= 0)
    if scheme in ("systematic", "residual", "stratified"):
        assert list(A) == list(range(N))


def test_schedule_at_threshold_zero_is_algorithm_one(orc):
    m = orc.Model(pf_inputs.lorenz63())
    xt, y = orc.simulate(m, 11, 3)
    N = 64
    X = orc.init(m, 5, 2, N)
    lz_a = lz_b = 0.0
    Xa, Xb = X.copy(), X.copy()
    lwc = np.zeros(N)
    for t in range(1, 4):
        ra = orc.filter_interval(m, 5, 2, t, Xa, y[t - 1], lz_a)
        rb = orc.filter_interval_sched(m, 5, 2, t, Xb, lwc, y[t - 1], lz_b, "multinomial", 0.0)
        assert rb["resampled"]
        assert np.array_equal(ra["A"], rb["A"])
        assert np.array_equal(ra["X"], rb["X"])
        assert np.array_equal(ra["lw"], rb["lw"])
        assert ra["logZ"] == rb["logZ"]
        assert np.array_equal(ra["mean_post"], rb["mean_est"])
        Xa, lz_a, Xb, lz_b, lwc = ra["X"], ra["logZ"], rb["X"], rb["logZ"], rb["lwc"]
        assert np.all(lwc == 0.0)


def test_never_resampling_is_sequential_importance_sampling(orc):
    # threshold 1e-300: ESS >= 1 > 1e-300 N, so the particles are never
    # resampled; the estimate is then sum_i W_i x_i / sum_i W_i with W_i the
    # product of every interval's likelihood, accumulated here with numpy
    # from the oracle's (pinned) propagation and log-likelihoods
    m = orc.Model(pf_inputs.lorenz63())
    _, y = orc.simulate(m, 12, 4)
    N = 32
    X = orc.init(m, 7, 1, N)
    Xs = X.copy()
    lwc = np.zeros(N)
    path = np.zeros(N)
    lz = 0.0
    lz_ref = 0.0
    for t in range(1, 5):
        r = orc.filter_interval_sched(m, 7, 1, t, X, lwc, y[t - 1], lz, "systematic", 1e-300)
        assert not r["resampled"]
        assert list(r["A"]) == list(range(N))
        Xs = orc.propagate(m, 7, 1, t, Xs)
        ll = orc.weights(m, Xs, y[t - 1])
        # evidence factor of the interval: sum_i W_{t-1,i} g_i / sum W_{t-1}
        prev = np.exp(path - path.max())
        path = path + ll
        cur = np.exp(path - path.max())
        lz_ref += (np.log(cur.sum()) + path.max()) - (np.log(prev.sum()) + (path - ll).max()) \
            - 0.5 * len(y[t - 1]) * np.log(2 * np.pi * 0.5)
        w = np.exp(path - path.max())
        ref = (w[:, None] * Xs).sum(0) / w.sum()
        assert np.allclose(r["X"], Xs, rtol=0, atol=0)
        assert np.allclose(r["mean_est"], ref, rtol=1e-12, atol=1e-12)
        assert r["logZ"] == pytest.approx(lz_ref, rel=1e-12, abs=1e-9)
        # carried weights normalised to mean weight 1
        assert np.mean(np.exp(r["lwc"])) == pytest.approx(1.0, rel=1e-12)
        X, lwc, lz = r["X"], r["lwc"], r["logZ"]


def _sched_run(orc, m, seed, N, y, scheme, thr):
    X = orc.init(m, seed, 0, N)
    lwc = np.zeros(N)
    lz = 0.0
    est = np.zeros((len(y), m.dx))
    n_rs = 0
    for t in range(1, len(y) + 1):
        r = orc.filter_interval_sched(m, seed, 0, t, X, lwc, y[t - 1], lz, scheme, thr)
        X, lwc, lz = r["X"], r["lwc"], r["logZ"]
        est[t - 1] = r["mean_est"]
        n_rs += r["resampled"]
    return est, lz, n_rs


@pytest.mark.parametrize("scheme", SCHEMES)
def test_ess_schedule_evidence_unbiased_ou(orc, scheme):
    spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 3, 3)
    _, _, ll = orc.kalman_ou(m, y[:, 0])
    R = 6000
    ratio = np.zeros(R)
    n_rs = 0
    for r in range(R):
        _, lz, k = _sched_run(orc, m, 700_000 + r, 8, y, scheme, 0.5)
        ratio[r] = np.exp(lz - ll)
        n_rs += k
    # the schedule both resamples and skips
    assert 0 < n_rs < 3 * R
    se = ratio.std() / np.sqrt(R)
    assert abs(ratio.mean() - 1.0) < 3 * se + 1e-3, (ratio.mean(), se)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_ess_schedule_tracks_kalman_mean(orc, scheme):
    spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 21, 30)
    km, kv, _ = orc.kalman_ou(m, y[:, 0])
    est, _, n_rs = _sched_run(orc, m, 4, 4000, y, scheme, 0.5)
    assert 0 < n_rs < 30
    err = est[:, 0] - km
    # Monte Carlo error of the posterior mean, a few posterior sd / sqrt(N)
    assert np.sqrt(np.mean(err ** 2)) < 6 * np.sqrt(np.mean(kv) / 4000), (err, kv)


# ------------------------------------------------------------------ the APF --
def _apf_run(orc, m, seed, N, y, scheme="multinomial"):
    X = orc.init(m, seed, 0, N)
    lwc = np.zeros(N)
    lz = 0.0
    est = np.zeros((len(y), m.dx))
    for t in range(1, len(y) + 1):
        r = orc.apf_interval(m, seed, 0, t, X, lwc, y[t - 1], lz, scheme)
        X, lwc, lz = r["X"], r["lwc"], r["logZ"]
        est[t - 1] = r["mean_w"]
    return est, lz


@pytest.mark.parametrize("scheme", ["multinomial", "residual"])
def test_apf_evidence_unbiased_ou(orc, scheme):
    # the auxiliary filter's two-stage estimate of p(y_t | y_1:t-1) keeps
    # E[G] = p(y_1:T) (Lemma 2 carries over): a wrong second-stage correction
    # (a missing pilot term, the pilot of slot k instead of its ancestor)
    # biases it
    spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 3, 3)
    _, _, ll = orc.kalman_ou(m, y[:, 0])
    R = 6000
    ratio = np.array([np.exp(_apf_run(orc, m, 800_000 + r, 8, y, scheme)[1] - ll)
                      for r in range(R)])
    se = ratio.std() / np.sqrt(R)
    assert abs(ratio.mean() - 1.0) < 3 * se + 1e-3, (ratio.mean(), se)
    # and its spread stays that of a proper importance weight (SE ~0.03 here);
    # a wrong correction makes the ratio heavy-tailed (planted: SE ~1e9)
    assert se < 0.1, se


def test_apf_tracks_kalman_mean(orc):
    spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 21, 30)
    km, kv, _ = orc.kalman_ou(m, y[:, 0])
    est, _ = _apf_run(orc, m, 4, 4000, y, "systematic")
    err = est[:, 0] - km
    assert np.sqrt(np.mean(err ** 2)) < 6 * np.sqrt(np.mean(kv) / 4000), (err, kv)


def test_apf_without_noise_has_flat_second_stage(orc):
    # with zero diffusion the pilot path is the particle's path, so the
    # second-stage weights g(y | x_k) / g(y | mu_{a_k}) are exactly 1
    spec = dict(pf_inputs.lorenz63(), noise_sd=(0.0, 0.0))
    m = orc.Model(spec)
    _, y = orc.simulate(m, 8, 2)
    N = 64
    X = orc.init(m, 3, 1, N)
    r = orc.apf_interval(m, 3, 1, 1, X, np.zeros(N), y[0], 0.0, "stratified")
    assert np.all(r["lw"] == 0.0)
    assert np.all(r["lwc"] == 0.0)
    assert r["ess"] == pytest.approx(N)
    # the estimate is the plain mean of the propagated first-stage selection
    ref = orc.mean(orc.propagate(m, 3, 1, 1, X[r["A"]]))
    assert np.allclose(r["mean_w"], ref, rtol=0, atol=1e-12)
