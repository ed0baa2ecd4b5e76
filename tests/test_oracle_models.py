"""Pins of the oracle's state-space models (CPU only).

Each pin comes from outside the oracle's own formulas: textbook fixed points
and phase-space contraction of Lorenz 63, scipy's image convolution for the
no-flux Laplacian, the cubic's known roots for the FitzHugh-Nagumo reaction,
the closed-form variance of Euler-Maruyama Brownian increments, and the
statistical independence of every noise variate the layout hands out.
"""
import numpy as np
import pytest
from scipy import ndimage

import pf_inputs


def test_lorenz_fixed_points(orc):
    m = orc.Model(pf_inputs.lorenz63())
    s, r, b = 10.0, 28.0, 8.0 / 3.0
    c = np.sqrt(b * (r - 1.0))
    for x in ([0.0, 0.0, 0.0], [c, c, r - 1.0], [-c, -c, r - 1.0]):
        assert np.allclose(orc.drift(m, x), 0.0, atol=1e-12)
    # a point off the attractor's fixed points moves
    assert np.linalg.norm(orc.drift(m, [1.0, 1.0, 1.0])) > 1.0


def test_lorenz_jacobian_trace(orc):
    # div f = -(s + 1 + b) everywhere (uniform phase-space contraction)
    m = orc.Model(pf_inputs.lorenz63())
    rng = np.random.default_rng(1)
    eps = 1e-6
    for _ in range(10):
        x = rng.normal(0, 10, 3)
        tr = 0.0
        for i in range(3):
            e = np.zeros(3)
            e[i] = eps
            tr += (orc.drift(m, x + e)[i] - orc.drift(m, x - e)[i]) / (2 * eps)
        assert tr == pytest.approx(-(10.0 + 1.0 + 8.0 / 3.0), abs=1e-6)


def test_lorenz_jacobian_at_origin(orc):
    # linearisation at the origin: [[-s, s, 0], [r, -1, 0], [0, 0, -b]]
    m = orc.Model(pf_inputs.lorenz63())
    eps = 1e-7
    Jm = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = eps
        Jm[:, j] = (orc.drift(m, e) - orc.drift(m, -e)) / (2 * eps)
    ref = np.array([[-10.0, 10.0, 0.0], [28.0, -1.0, 0.0], [0.0, 0.0, -8.0 / 3.0]])
    assert np.allclose(Jm, ref, atol=1e-6)


def test_em_step_noise_scaling(orc):
    # at a fixed point the deterministic part vanishes: x' - x = sd sqrt(h) z
    m = orc.Model(pf_inputs.lorenz63())
    z = np.array([0.3, -1.2, 2.0])
    x0 = np.zeros(3)
    assert np.allclose(orc.em_step(m, x0, z) - x0, 0.5 * np.sqrt(1e-3) * z, atol=1e-15)


def test_laplacian_matches_scipy_nearest(orc):
    # edge replication makes the outside neighbour equal to the node itself,
    # i.e. exactly the truncated (no-flux) neighbourhoods of the grid.
    rng = np.random.default_rng(3)
    for J in (2, 3, 7, 20, 40):
        v = rng.normal(size=(J, J))
        k = np.array([[0.0, 1.0, 0.0], [1.0, -4.0, 1.0], [0.0, 1.0, 0.0]])
        ref = ndimage.convolve(v, k, mode="nearest")
        assert np.allclose(orc.laplacian(v), ref, atol=1e-12)


def test_laplacian_impulse_and_conservation(orc):
    J = 6
    for (i, j), centre in (((0, 0), -2), ((0, 3), -3), ((3, 0), -3), ((3, 3), -4), ((5, 5), -2)):
        v = np.zeros((J, J))
        v[i, j] = 1.0
        lap = orc.laplacian(v)
        assert lap[i, j] == centre
        assert lap.sum() == pytest.approx(0.0, abs=1e-14)
    assert np.allclose(orc.laplacian(np.full((J, J), 2.5)), 0.0)


def test_fhn_reaction_roots_and_recovery(orc):
    spec = pf_inputs.fhn(J=4)
    m = orc.Model(spec)
    nn = 16
    for v0 in (0.0, 0.1, 1.0):
        x = np.concatenate([np.full(nn, v0), np.zeros(nn)])
        f = orc.drift(m, x)
        assert np.allclose(f[:nn], 0.0, atol=1e-15)
    # recovery: w-nullcline at w = v / gamma, slope eps
    x = np.concatenate([np.full(nn, 0.4), np.full(nn, 0.8)])
    f = orc.drift(m, x)
    assert np.allclose(f[nn:], 0.0, atol=1e-15)
    x = np.concatenate([np.full(nn, 0.4), np.zeros(nn)])
    assert np.allclose(orc.drift(m, x)[nn:], 0.01 * 0.4)
    # v-derivative of the cubic at 0 equals -a (excitable rest state)
    e = 1e-7
    xp = np.concatenate([np.full(nn, e), np.zeros(nn)])
    xm = np.concatenate([np.full(nn, -e), np.zeros(nn)])
    d = (orc.drift(m, xp)[:nn] - orc.drift(m, xm)[:nn]) / (2 * e)
    assert np.allclose(d, -0.1, atol=1e-6)


def test_fhn_coupling_enters_v_only(orc):
    spec = pf_inputs.fhn(J=5)
    m = orc.Model(spec)
    rng = np.random.default_rng(4)
    v = rng.normal(size=(5, 5)) * 0.001
    x = np.concatenate([v.ravel(), np.zeros(25)])
    f = orc.drift(m, x)
    lin = -0.1 * v.ravel() + 0.5 * ndimage.convolve(
        v, np.array([[0, 1, 0], [1, -4, 1], [0, 1, 0]], float), mode="nearest").ravel()
    # near v = 0 the cubic is -a v + O(v^2); coupling is D * lap
    assert np.allclose(f[:25], lin, atol=2e-5)


def test_brownian_variance_closed_form(orc):
    # OU with theta = 0 is Brownian motion: Var x_{nh} = n h sd^2
    spec = pf_inputs.ou1d(theta=0.0, sd=1.3, h=0.02, S=25, prior_sd=1e-300, prior_mean=0.0)
    m = orc.Model(spec)
    X = np.zeros((20000, 1))
    X = orc.propagate(m, 9, 0, 1, X)
    var = X[:, 0].var()
    expect = 25 * 0.02 * 1.3**2
    assert var == pytest.approx(expect, rel=5 * np.sqrt(2 / 20000))


def test_step_noise_independent_across_steps_and_components(orc):
    # every (step, component) gets its own standard normal: the empirical
    # correlation of 8 consecutive steps x 3 components is the identity.
    m = orc.Model(pf_inputs.lorenz63())
    n_p = 4000
    Z = np.zeros((n_p, 8 * 3))
    for p in range(n_p):
        Z[p] = np.concatenate([orc.step_noise(m, 1, orc.P_PROP, p, 2, n) for n in range(8)])
    cm = np.corrcoef(Z.T)
    assert np.max(np.abs(cm - np.eye(24))) < 6.0 / np.sqrt(n_p)
    assert np.allclose(Z.var(0), 1.0, atol=6 * np.sqrt(2 / n_p))


def test_grid_noise_layout(orc):
    spec = pf_inputs.fhn(J=4)
    m = orc.Model(spec)
    z = orc.step_noise(m, 5, orc.P_PROP, 3, 1, 7)
    k = orc.key(5)
    for p in range(8):
        q = orc.normals4([3, 1, 7, (orc.P_PROP << 24) | p], k)
        assert z[2 * p] == q[0] and z[16 + 2 * p] == q[1]
        assert z[2 * p + 1] == q[2] and z[16 + 2 * p + 1] == q[3]


def test_loglik_hand_values(orc):
    m = orc.Model(pf_inputs.lorenz63())
    # residuals (2-1, 5-3) = (1, 2): -(1 + 4) / (2 * 0.5) = -5
    assert orc.loglik(m, [1.0, 2.0, 3.0], [2.0, 5.0]) == -5.0
    assert orc.loglik(m, [np.nan, 2.0, 3.0], [2.0, 5.0]) == -np.inf


def test_paper_lorenz_observation_and_prior(orc):
    # the paper's Lorenz experiment: y_t = X_{1,100t} + V_t with var(V) = 1/2
    # (eqObservLorenz), so a particle's log-weight is -(y - x1)^2 and does not
    # see x2, x3; the prior is N(x*, 10 I) (Sec. 4.1)
    from scipy import stats
    m = orc.Model(pf_inputs.lorenz63_paper())
    X = np.array([[1.0, 2.0, 3.0], [1.0, -7.0, 40.0], [3.5, 0.0, 0.0]])
    lw = orc.weights(m, X, np.array([2.0]))
    assert lw == pytest.approx([-1.0, -1.0, -2.25], abs=1e-15)
    n = 20000
    x0 = orc.init(m, 5, 0, n)
    dof = n - 1
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], dof)
    for c, mu in enumerate([-10.2410, -1.3984, 23.6752]):
        v = np.var(x0[:, c], ddof=1)
        assert lo * 10.0 / dof < v < hi * 10.0 / dof, (c, v)
        assert abs(np.mean(x0[:, c]) - mu) < 5 * np.sqrt(10.0 / n)
