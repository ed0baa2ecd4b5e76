"""Pins of the oracle's learned-proposal functions (CPU only).

The learned proposal adds a drift correction u_theta to every Euler-Maruyama
increment and multiplies each particle's weight by the exact ratio of the
model and proposal increment densities; the consistency of such weighted
proposals is the importance-function extension the paper's closing remarks
(Sec. 6) point to.  Nothing here uses the oracle to check itself:

* the MLP forward pass and its gradient against torch's own Linear/ReLU
  modules and autograd in float64, and against central finite differences;
* bfloat16 rounding against torch's float32 -> bfloat16 cast;
* the 22 FH-N features against hand-derived values (edge replication,
  nearest observation with ties to the lower index, tau, offsets);
* u = 0 reproduces the bootstrap filter bit for bit;
* the increment-density ratio has mean one under the proposal;
* with an arbitrary fixed u the filter still tracks the exact Kalman mean and
  its evidence estimate stays unbiased (Lemma 2), which pins the ratio's sign
  and both of its terms;
* the closed-form minimiser of the regression objective on the OU model
  against a Monte Carlo regression run with numpy's own generator;
* Adam against torch.optim.Adam;
* the training paths: every increment of a trajectory is its Euler step with
  the documented noise, which is N(0, 1) and independent across the run,
  trajectory and minibatch streams.
"""
import numpy as np
import pytest
import torch

import pf_inputs

H = 64


def _rand_params(orc, rng, in_dim, out_dim, scale=0.3):
    p = np.zeros(orc.mlp_nparams(in_dim, out_dim))
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, in_dim, out_dim)
    W1[:] = rng.standard_normal(W1.shape) * scale
    b1[:] = rng.standard_normal(b1.shape) * 0.1
    W2[:] = rng.standard_normal(W2.shape) * scale / 2
    b2[:] = rng.standard_normal(b2.shape) * 0.1
    W3[:] = rng.standard_normal(W3.shape) * scale / 2
    b3[:] = rng.standard_normal(b3.shape) * 0.1
    return p


def _torch_mlp(orc, p, in_dim, out_dim):
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, in_dim, out_dim)
    net = torch.nn.Sequential(torch.nn.Linear(in_dim, H), torch.nn.ReLU(),
                              torch.nn.Linear(H, H), torch.nn.ReLU(),
                              torch.nn.Linear(H, out_dim)).double()
    with torch.no_grad():
        for lin, W, b in zip((net[0], net[2], net[4]), (W1, W2, W3), (b1, b2, b3)):
            lin.weight.copy_(torch.from_numpy(W.copy()))
            lin.bias.copy_(torch.from_numpy(b.copy()))
    return net


@pytest.mark.parametrize("in_dim,out_dim", [(20, 2), (3, 1)])
def test_mlp_forward_matches_torch(orc, in_dim, out_dim):
    rng = np.random.default_rng(in_dim)
    p = _rand_params(orc, rng, in_dim, out_dim)
    x = rng.standard_normal((50, in_dim))
    out, _, _ = orc.mlp_forward(p, x, out_dim)
    ref = _torch_mlp(orc, p, in_dim, out_dim)(torch.from_numpy(x)).detach().numpy()
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("in_dim,out_dim", [(20, 2), (3, 1)])
def test_mlp_gradient_matches_autograd(orc, in_dim, out_dim):
    rng = np.random.default_rng(100 + in_dim)
    p = _rand_params(orc, rng, in_dim, out_dim)
    X = rng.standard_normal((16, in_dim))
    T = rng.standard_normal((16, out_dim))
    loss, g = orc.mlp_loss_grad(p, X, T)
    net = _torch_mlp(orc, p, in_dim, out_dim)
    L = ((net(torch.from_numpy(X)) - torch.from_numpy(T)) ** 2).sum(1).mean()
    L.backward()
    ref = np.concatenate([t.grad.numpy().ravel() for t in
                          (net[0].weight, net[0].bias, net[2].weight, net[2].bias,
                           net[4].weight, net[4].bias)])
    assert abs(loss - L.item()) <= 1e-12 * abs(L.item())
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-13)


def test_mlp_gradient_matches_central_differences(orc):
    rng = np.random.default_rng(7)
    in_dim, out_dim = 20, 2
    p = _rand_params(orc, rng, in_dim, out_dim)
    X = rng.standard_normal((8, in_dim))
    T = rng.standard_normal((8, out_dim))
    _, g = orc.mlp_loss_grad(p, X, T)
    # no pre-activation may sit within the step of a ReLU kink
    eps = 1e-6
    fd = np.zeros_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = eps
        fd[k] = (orc.mlp_loss_grad(p + e, X, T)[0] - orc.mlp_loss_grad(p - e, X, T)[0]) / (2 * eps)
    err = np.linalg.norm(fd - g) / np.linalg.norm(g)
    assert err < 1e-6, err


def test_bf16_rounding_matches_torch(orc):
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(4000) * np.exp(rng.uniform(-20, 20, 4000))).astype(np.float32)
    # exact ties: bfloat16 values plus half a unit in their last place
    b = torch.from_numpy(x[:500].copy()).to(torch.bfloat16).to(torch.float64).numpy()
    ties = (b + np.sign(b) * 2.0 ** (np.floor(np.log2(np.abs(b))) - 8)).astype(np.float32)
    vals = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, 1.00390625, 1.01171875])])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    got = orc.bf16(vals.astype(np.float64))
    assert np.array_equal(got, ref)


def test_mlp_bf16_mode_semantics(orc):
    """bf16 mode: inputs and parameters rounded, hidden activations rounded
    to the nearest bfloat16 after the ReLU, the output layer exact on them."""
    rng = np.random.default_rng(11)
    in_dim, out_dim = 20, 2
    p = _rand_params(orc, rng, in_dim, out_dim)
    x = rng.standard_normal((40, in_dim))
    out, h1, h2 = orc.mlp_forward(p, x, out_dim, bf16_mode=True)
    # rounding of float64 values is pinned by the float32 cases above
    pq, xq = orc.bf16(p), orc.bf16(x)
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(pq, in_dim, out_dim)
    for h in (h1, h2):
        hq = torch.from_numpy(h).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(h, hq), "hidden activations are bfloat16 values"
    a1 = np.maximum(xq @ W1.T + b1, 0.0)
    # round to nearest with 8 significant bits: within 2^-8 relative
    assert np.all(np.abs(h1 - a1) <= 2.0 ** -8 * np.abs(a1))
    a2 = np.maximum(h1 @ W2.T + b2, 0.0)
    assert np.all(np.abs(h2 - a2) <= 2.0 ** -8 * np.abs(a2) * (1 + 1e-12))
    assert np.allclose(out, h2 @ W3.T + b3, rtol=1e-12, atol=1e-12)


def test_nearest_observation_and_features(orc):
    spec = pf_inputs.fhn(20)
    m = orc.Model(spec)
    J = 20
    near = orc.nearest_obs(m)
    obs = list(spec["obs_idx"])
    assert obs[0] == 2 * J + 2 and obs[-1] == 18 * J + 18
    assert near[0] == 0                       # (0,0) -> (2,2)
    assert near[4 * J + 4] == 0               # equidistant from four: lowest index
    assert near[19 * J + 19] == len(obs) - 1  # (19,19) -> (18,18)
    assert near[2 * J + 6] == 1               # on the observation (2,6)
    assert near[2 * J + 4] == 0               # tie between (2,2) and (2,6)
    assert near[9 * J + 17] == obs.index(10 * J + 18)
    nn = J * J
    x = np.concatenate([np.arange(nn, dtype=np.float64), 1000.0 + np.arange(nn)])
    y = np.arange(len(obs), dtype=np.float64) * 0.5
    f = orc.fhn_features(m, x, y, k=0, nodes=[0, 5 * J + 19, 7 * J + 3])
    assert list(f[0, :9]) == [0, 0, 1, 0, 0, 1, 20, 20, 21]
    assert list(f[0, 9:18]) == [1000 + v for v in [0, 0, 1, 0, 0, 1, 20, 20, 21]]
    assert f[0, 18] == y[0] - obs[0]
    assert f[0, 19] == 1.0
    c = 5 * J + 19
    assert list(f[1, :9]) == [c - J - 1, c - J, c - J, c - 1, c, c, c + J - 1, c + J, c + J]
    o = near[c]
    assert f[1, 18] == y[o] - obs[o]
    c = 7 * J + 3
    assert list(f[2, :9]) == [c - J - 1, c - J, c - J + 1, c - 1, c, c + 1, c + J - 1, c + J,
                              c + J + 1]
    g = orc.fhn_features(m, x, y, k=19, nodes=[0])
    assert g[0, 19] == 1.0 / 20
    # offsets of the nearest observation, halved: (0,0) -> (2,2); (5,19) -> (6,18)
    assert list(f[0, 20:]) == [1.0, 1.0]
    assert list(f[1, 20:]) == [0.5, -0.5]
    assert list(f[2, 20:]) == [-0.5, -0.5]  # (7,3) -> (6,2)


@pytest.mark.parametrize("which", ["fhn", "ou"])
def test_zero_network_is_the_bootstrap_filter(orc, which):
    if which == "fhn":
        spec = pf_inputs.fhn(20)
        in_dim, out_dim, N = 22, 2, 3
    else:
        spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)
        in_dim, out_dim, N = 3, 1, 64
    m = orc.Model(spec)
    xt, y = orc.simulate(m, 5, 3)
    p = np.zeros(orc.mlp_nparams(in_dim, out_dim))
    X = orc.init(m, 9, 2, N)
    a, b = X.copy(), X.copy()
    lza = lzb = 0.0
    for t in range(1, 4):
        ra = orc.filter_interval(m, 9, 2, t, a, y[t - 1], lza)
        rb = orc.filter_interval_learned(m, p, 9, 2, t, b, y[t - 1], lzb)
        for k in ("X", "lw", "A", "mean_post", "mean_w"):
            assert np.array_equal(ra[k], rb[k]), k
        assert ra["logZ"] == rb["logZ"]
        a, b, lza, lzb = ra["X"], rb["X"], ra["logZ"], rb["logZ"]
    Xp, dlw = orc.propagate_learned(m, p, 9, 2, 4, a, y[2])
    assert np.array_equal(Xp, orc.propagate(m, 9, 2, 4, a))
    assert np.all(dlw == 0.0)


def _ou_spec():
    return pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.05)


def test_increment_ratio_has_unit_mean(orc):
    """E_q[p/q] = 1 for the path density ratio; a wrong sign or a missing
    factor 1/2 on the u^2 term moves the mean by many standard errors."""
    m = orc.Model(_ou_spec())
    rng = np.random.default_rng(5)
    p = _rand_params(orc, rng, 3, 1, scale=1.0)
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, 3, 1)
    b3[:] = 2.0  # u around 2: per interval S c^2 u^2 / 2 = 0.2 with c = sqrt(h)/sd
    N = 20000
    X = np.zeros((N, 1))
    _, dlw = orc.propagate_learned(m, p, 21, 0, 1, X, np.array([0.7]), bf16_mode=False)
    r = np.exp(dlw)
    se = r.std(ddof=1) / np.sqrt(N)
    assert abs(r.mean() - 1.0) < 4 * se, (r.mean(), se)
    assert np.mean(dlw) < -0.1  # the correction is not trivially zero


def test_fixed_network_tracks_kalman_and_keeps_evidence_unbiased(orc):
    m = orc.Model(_ou_spec())
    rng = np.random.default_rng(8)
    p = _rand_params(orc, rng, 3, 1, scale=0.8)
    T = 10
    _, y = orc.simulate(m, 44, T)
    kmean, _, _ = orc.kalman_ou(m, y[:, 0])
    est, _, _, _ = orc.run_ensemble_learned(m, p, 3, 8, 512, y, bf16_mode=False)
    est_b, _, _, _ = orc.run_ensemble(m, 3, 8, 512, y)
    mse_l = np.mean((est[:, 0] - kmean) ** 2)
    mse_b = np.mean((est_b[:, 0] - kmean) ** 2)
    # the posterior sd is about 0.2; an inconsistent weight biases by that order
    assert mse_l < 4 * mse_b + 1e-4, (mse_l, mse_b)
    assert mse_l < 2e-3
    # Lemma 2: E[G_T] = p(y_{1:T}), over many small filters
    T2 = 3
    _, y2 = orc.simulate(m, 45, T2)
    lz = np.concatenate([orc.run_ensemble_learned(m, p, s, 50, 32, y2, bf16_mode=False)[2]
                         for s in range(8)])
    _, _, exact = orc.kalman_ou(m, y2[:, 0])
    r = np.exp(lz - exact)
    se = r.std(ddof=1) / np.sqrt(r.size)
    assert abs(r.mean() - 1.0) < 3 * se + 1e-3, (r.mean(), se)


def test_ou_optimal_drift_by_monte_carlo(orc):
    """(sd/sqrt(h)) E[z_k | x_k = x, y], estimated by a least-squares fit of
    the scaled noise on y over simulated intervals (numpy's generator)."""
    spec = _ou_spec()
    m = orc.Model(spec)
    theta, sd, h, S, R = 1.0, 1.0, 0.01, 10, 0.05
    rng = np.random.default_rng(123)
    n = 400_000
    for k, x0 in ((0, 0.4), (6, -1.1), (9, 0.0)):
        x = np.full(n, x0)
        z = rng.standard_normal((S - k, n))
        for j in range(S - k):
            x = x + h * (-theta * x) + sd * np.sqrt(h) * z[j]
        y = x + np.sqrt(R) * rng.standard_normal(n)
        target = sd / np.sqrt(h) * z[0]
        A = np.stack([np.ones(n), y], 1)
        coef, *_ = np.linalg.lstsq(A, target, rcond=None)
        resid = target - A @ coef
        for yq in (-0.5, 0.3, 1.0):
            pred = coef[0] + coef[1] * yq
            # standard error of the fitted mean at yq
            Xi = np.linalg.inv(A.T @ A)
            v = np.array([1.0, yq])
            se = np.sqrt(resid.var() * v @ Xi @ v)
            assert abs(pred - orc.ou_optimal_u(m, x0, yq, k)) < 4 * se + 1e-9, (k, yq)


def test_learned_fhn_interval_is_finite_and_resamples(orc):
    spec = pf_inputs.fhn(20)
    m = orc.Model(spec)
    rng = np.random.default_rng(2)
    p = _rand_params(orc, rng, 22, 2, scale=0.05)
    _, y = orc.simulate(m, 3, 1)
    X = orc.init(m, 4, 0, 3)
    r = orc.filter_interval_learned(m, p, 4, 0, 1, X, y[0])
    assert np.all(np.isfinite(r["X"])) and np.all(np.isfinite(r["lw"]))
    assert np.all(np.diff(r["A"]) >= 0)
    Xp, dlw = orc.propagate_learned(m, p, 4, 0, 1, X, y[0])
    assert np.all(dlw != 0.0)
    assert np.array_equal(r["lw"], orc.weights(m, Xp, y[0]) + dlw)


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(4)
    p0 = rng.standard_normal(50)
    grads = rng.standard_normal((7, 50))
    p, mo, ve = p0.copy(), np.zeros(50), np.zeros(50)
    w = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        orc.adam_step(p, grads[t - 1], mo, ve, 1e-2, 0.9, 0.999, 1e-8, t)
        w.grad = torch.from_numpy(grads[t - 1].copy())
        opt.step()
    assert np.allclose(p, w.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_training_paths_are_model_paths(orc):
    spec = pf_inputs.fhn(20)
    m = orc.Model(spec)
    starts = orc.train_run(m, 3, 2, 3)
    assert starts.shape == (3, 800) and np.all(np.isfinite(starts))
    assert not np.allclose(starts[0], starts[1])
    traj, y, z = orc.train_trajectory(m, 3, 5, starts[1])
    assert np.array_equal(traj[0], starts[1])
    for k in range(spec["S"] - 1):
        assert np.allclose(orc.em_step(m, traj[k], z[k]), traj[k + 1], rtol=0, atol=0)
    # the noise of the trajectory, the run and the step-0 bootstrap draw are
    # distinct streams of standard normals
    zz = z.ravel()
    assert abs(zz.mean()) < 4 / np.sqrt(zz.size) and abs(zz.var() - 1) < 0.05
    zb = orc.step_noise(m, 3, orc.P_PROP, 5, 0, 0)
    assert abs(np.corrcoef(z[0], zb)[0, 1]) < 0.1
    # y is the observation of the state after the last step
    xS = orc.em_step(m, traj[-1], z[-1])
    r = (y - xS[m.obs_idx]) / np.sqrt(spec["obs_var"])
    assert np.all(np.abs(r) < 6)
    tiles = [orc.train_tile(m, 3, 100, 7, b) for b in range(2000)]
    rs, ks, ns = map(np.array, zip(*tiles))
    assert rs.min() >= 0 and rs.max() < 100 and ks.min() >= 0 and ks.max() < 20
    assert np.all(ns % 16 == 0) and ns.max() <= 400 - 16
    assert len(set(ks)) == 20 and len(set(ns)) == 25
