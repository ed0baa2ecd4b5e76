"""GPU training of the learned proposal (MI355X only).

* The minibatch gradient (MFMA forward, hand-written backward, MFMA weight
  gradients) against the oracle's FP64 gradient at the bfloat16-rounded
  parameters: relative L2 error below 1e-2 and cosine above 0.999 (the GPU
  rounds hidden activations and layer errors to bfloat16, about 2^-9
  relative each), for explicit rows and for the FH-N minibatches the
  trainer draws from its trajectories (features and targets built on the
  GPU; the oracle builds the same rows from its own trajectories).
* Adam against the oracle's FP64 Adam.
* The training paths (long runs, trajectories, observations) against the
  oracle's, to the bootstrap state tolerance summed over the intervals.
* Training: on the OU model the network trained on the GPU approaches the
  closed-form optimal drift (R^2 > 0.9); on FH-N 20 x 20 training lowers the
  regression loss on trajectories it has not seen, and the trained proposal
  beats the bootstrap filter at the same N.
"""
import numpy as np
import pytest

import pf_inputs
from pf_testlib import assert_rel_close

pytestmark = pytest.mark.gpu

F20 = pf_inputs.fhn(20)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def pf(torch_mod):
    import paper_1407_8071_amd as pf
    pf.lib()
    return pf


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _he_init(orc, rng, in_dim, out_dim, scale=1.0):
    p = np.zeros(orc.mlp_nparams(in_dim, out_dim))
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, in_dim, out_dim)
    W1[:] = rng.standard_normal(W1.shape) * np.sqrt(2 / in_dim) * scale
    W2[:] = rng.standard_normal(W2.shape) * np.sqrt(2 / 64) * scale
    W3[:] = rng.standard_normal(W3.shape) * np.sqrt(1 / 64) * scale
    b1[:] = rng.standard_normal(64) * 0.05
    b2[:] = rng.standard_normal(64) * 0.05
    b3[:] = rng.standard_normal(out_dim) * 0.05
    return p.astype(np.float32).astype(np.float64)


def _compare_grad(got, ref):
    got = np.asarray(got, np.float64)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    cos = got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref))
    assert rel < 1e-2 and cos > 0.999, (rel, cos)


@pytest.mark.parametrize("in_dim,out_dim,rows", [(20, 2, 1000), (3, 1, 77), (20, 2, 16 * 300)])
def test_gradient_matches_oracle(pf, orc, torch_mod, in_dim, out_dim, rows):
    rng = np.random.default_rng(rows)
    p = _he_init(orc, rng, in_dim, out_dim)
    X = orc.bf16(rng.standard_normal((rows, in_dim)).astype(np.float32))
    T = rng.standard_normal((rows, out_dim)).astype(np.float32).astype(np.float64)
    loss, g = pf.mlp_loss_grad(_dev(p), _dev(X), _dev(T))
    rloss, rg = orc.mlp_loss_grad(orc.bf16(p), X, T)
    assert abs(loss.item() - rloss) <= 1e-2 * rloss
    _compare_grad(g.cpu().numpy(), rg)


def test_adam_matches_oracle(pf, orc, torch_mod):
    rng = np.random.default_rng(9)
    n = 5634
    p = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    mo = (rng.standard_normal(n) * 0.1).astype(np.float32).astype(np.float64)
    ve = (rng.random(n) * 0.01).astype(np.float32).astype(np.float64)
    g = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    dp, dm, dv = _dev(p), _dev(mo), _dev(ve)
    m0, v0 = mo.copy(), ve.copy()
    pf.adam_step(dp, _dev(g), dm, dv, 1e-3, 0.9, 0.999, 1e-8, 3)
    orc.adam_step(p, g, mo, ve, 1e-3, 0.9, 0.999, 1e-8, 3)
    # FP32: the coefficients and each product and sum carry a relative
    # rounding of 2^-24, so each moment is within a few units of 2^-24 of
    # the sizes of its two terms; the update within that of lr
    u = 2.0 ** -24
    assert np.all(np.abs(dm.cpu().numpy() - mo) <= 4 * u * (0.9 * np.abs(m0) + 0.1 * np.abs(g)))
    assert np.all(np.abs(dv.cpu().numpy() - ve) <= 4 * u * (0.999 * v0 + 0.001 * g * g))
    assert np.all(np.abs(dp.cpu().numpy() - p) <= 4 * u * np.abs(p) + 1e-3 * 1e-5)


def _oracle_training_set(orc, m, seed, n_runs, run_len):
    trajs, ys, zs = [], [], []
    for q in range(n_runs):
        starts = orc.train_run(m, seed, q, run_len)
        for j in range(run_len):
            tr, y, z = orc.train_trajectory(m, seed, q * run_len + j, starts[j])
            trajs.append(tr)
            ys.append(y)
            zs.append(z)
    return np.array(trajs), np.array(ys), np.array(zs)


def test_training_paths_match_oracle(pf, orc, torch_mod):
    n_runs, run_len, seed = 2, 2, 11
    tr = pf.Trainer(F20, n_runs, run_len, batch_tiles=4, seed=seed)
    tr.data()
    starts, traj, ys = [t.cpu().numpy() for t in tr.buffers()]
    m = orc.Model(F20)
    otraj, oys, _ = _oracle_training_set(orc, m, seed, n_runs, run_len)
    for q in range(n_runs):
        ostarts = orc.train_run(m, seed, q, run_len)
        for j in range(run_len):
            # j + 1 intervals from the prior draw: the one-interval bound per interval
            assert_rel_close(starts[q * run_len + j], ostarts[j], floor=0.1, rel=1e-5 * (j + 1),
                             what="start states")
    for r in range(n_runs * run_len):
        nint = r % run_len + 2
        assert_rel_close(traj[r], otraj[r], floor=0.1, rel=1e-5 * nint, what="trajectories")
        assert_rel_close(ys[r], oys[r], floor=0.1, rel=1e-5 * nint, what="observations")


def test_fhn_minibatch_gradient_matches_oracle(pf, orc, torch_mod):
    n_runs, run_len, seed, tiles = 2, 3, 5, 6
    tr = pf.Trainer(F20, n_runs, run_len, batch_tiles=tiles, seed=seed)
    tr.data()
    m = orc.Model(F20)
    otraj, oys, ozs = _oracle_training_set(orc, m, seed, n_runs, run_len)
    rng = np.random.default_rng(2)
    p = _he_init(orc, rng, 22, 2, scale=0.5)
    nn = 400
    ts = np.array(F20["noise_sd"]) / np.sqrt(F20["h"])
    for step in (1, 7):
        X, T = [], []
        for b in range(tiles):
            r, k, n0 = orc.train_tile(m, seed, n_runs * run_len, step, b)
            nodes = np.arange(n0, n0 + 16)
            X.append(orc.fhn_features(m, otraj[r][k], oys[r], k, list(nodes)))
            T.append(np.stack([ozs[r][k][nodes] * ts[0], ozs[r][k][nn + nodes] * ts[1]], 1))
        X, T = np.concatenate(X), np.concatenate(T)
        rloss, rg = orc.mlp_loss_grad(orc.bf16(p), orc.bf16(X), T)
        loss, g = tr.grad(_dev(p), step)
        assert abs(loss.item() - rloss) <= 1e-2 * rloss
        _compare_grad(g.cpu().numpy(), rg)


def _ou_rows(n_int, seed, theta=1.0, sd=1.0, h=0.01, S=10, R=0.05):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n_int) * np.sqrt(sd ** 2 / (2 * theta))
    xs, z = np.zeros((S, n_int)), rng.standard_normal((S, n_int))
    for k in range(S):
        xs[k] = x
        x = x + h * (-theta * x) + sd * np.sqrt(h) * z[k]
    y = x + np.sqrt(R) * rng.standard_normal(n_int)
    k = np.repeat(np.arange(S)[:, None], n_int, 1)
    X = np.stack([xs.ravel(), (y[None, :] - xs).ravel(), ((S - k) / S).ravel()], 1)
    return X, (sd / np.sqrt(h) * z).ravel()[:, None]


def test_training_learns_the_optimal_ou_drift(pf, orc, torch_mod):
    """Regression onto (sd/sqrt(h)) z has the minimiser (sd/sqrt(h)) E[z | x, y, k],
    which is closed-form for the OU model; the GPU-trained network must
    explain 90% of its variance on a grid of states, observations and steps."""
    import torch
    spec = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.05)
    m = orc.Model(spec)
    X, T = _ou_rows(20000, 1)
    perm = np.random.default_rng(0).permutation(X.shape[0])
    Xd, Td = _dev(X[perm]), _dev(T[perm])
    p = _dev(_he_init(orc, np.random.default_rng(0), 3, 1))
    mo = torch.zeros_like(p)
    ve = torch.zeros_like(p)
    B, nb = 4096, X.shape[0] // 4096
    for t in range(1, 1601):
        b = (t - 1) % nb
        _, g = pf.mlp_loss_grad(p, Xd[b * B:(b + 1) * B], Td[b * B:(b + 1) * B])
        pf.adam_step(p, g, mo, ve, 1e-3, 0.9, 0.999, 1e-8, t)
    grid = [(x, y, k) for x in np.linspace(-1, 1, 9) for y in np.linspace(-1.5, 1.5, 9)
            for k in range(10)]
    Xg = np.array([[x, y - x, (10 - k) / 10] for x, y, k in grid])
    ustar = np.array([orc.ou_optimal_u(m, x, y, k) for x, y, k in grid])
    u, _, _ = orc.mlp_forward(p.cpu().numpy().astype(np.float64), Xg, 1, bf16_mode=True)
    r2 = 1 - np.sum((u[:, 0] - ustar) ** 2) / np.sum((ustar - ustar.mean()) ** 2)
    print(f"OU optimal-drift R^2 = {r2:.4f}")
    assert r2 > 0.9, r2


def _zero_output_init(orc, rng):
    """He-initialised hidden layers, zero output layer: training starts from
    the bootstrap proposal."""
    p = _he_init(orc, rng, 22, 2)
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, 22, 2)
    b1[:] = b2[:] = 0.0
    W3[:] = 0.0
    b3[:] = 0.0
    return p


@pytest.fixture(scope="module")
def trained_fhn20(pf, orc, torch_mod):
    """FH-N 20 x 20 proposal trained on 1e4 model trajectories (100 runs of
    100 intervals), 6000 Adam steps of 4096 tiles with the learning rate
    stepped down 3e-4, 1e-4, 3e-5."""
    tr = pf.Trainer(F20, 100, 100, batch_tiles=4096, seed=21)
    tr.data()
    p = _dev(_zero_output_init(orc, np.random.default_rng(1)))
    losses = []
    for n, lr in ((2000, 3e-4), (2000, 1e-4), (2000, 3e-5)):
        tr.desc.lr = lr
        losses.append(tr.steps(p, n).cpu().numpy())
    assert np.all(np.isfinite(np.concatenate(losses)))
    assert np.all(np.isfinite(p.cpu().numpy()))
    return p


def test_fhn_training_lowers_unseen_loss(pf, orc, torch_mod, trained_fhn20):
    import torch
    p = trained_fhn20
    held = pf.Trainer(F20, 10, 50, batch_tiles=1024, seed=99)
    held.data()
    zero = torch.zeros_like(p)
    d = []
    for s in range(1, 31):
        lt, _ = held.grad(p, s)
        l0, _ = held.grad(zero, s)
        d.append(lt.item() - l0.item())
    d = np.array(d)
    se = d.std(ddof=1) / np.sqrt(d.size)
    print(f"FH-N held-out loss change {d.mean():.3e} +- {se:.1e} (zero-network loss {l0.item():.4f})")
    assert d.mean() < -3 * se


def test_learned_proposal_gain_over_bootstrap(pf, orc, torch_mod, trained_fhn20):
    """What the trained network gains: on the same observations and seeds,
    the learned filter's MSE of v against the truth is below the bootstrap
    filter's at the same N (paired over 8 truths, by more than 2 standard
    errors) and its ESS is higher; the bootstrap filter with 4N particles is
    printed beside them."""
    import torch
    m = orc.Model(F20)
    T, M, N = 40, 8, 128

    def run(y, xt, learned, n, seed):
        f = pf.ParticleFilter([F20], [(0, M, n, seed, pf.ENS_LEARNED if learned else 0)],
                              fused=True)
        if learned:
            f.set_proposal(0, trained_fhn20)
        yd = _dev(y)
        est = np.zeros((T, F20["dx"]))
        ess = np.zeros(T)
        for t in range(T):
            f.step(yd[t])
            est[t] = f.estimate()[0].cpu().numpy()
            st = f.get_filter_stats(0).cpu().numpy().reshape(M, 4)
            ess[t] = np.mean(st[:, 1] ** 2 / st[:, 2])
        return np.mean((est[:, :400] - xt[1:, :400]) ** 2), ess.mean()

    rows = []
    for s in range(8):
        xt, y = orc.simulate(m, 7000 + s, T)
        rows.append(run(y, xt, False, N, 10 + s) + run(y, xt, True, N, 10 + s) +
                    run(y, xt, False, 4 * N, 10 + s))
    r = np.array(rows)
    d = r[:, 2] - r[:, 0]
    se = d.std(ddof=1) / np.sqrt(d.size)
    print(f"MSE(v): bootstrap N={N} {r[:, 0].mean():.5f}, learned N={N} {r[:, 2].mean():.5f}, "
          f"bootstrap N={4 * N} {r[:, 4].mean():.5f}; ESS {r[:, 1].mean():.2f} / "
          f"{r[:, 3].mean():.2f} / {r[:, 5].mean():.2f}; paired gain {d.mean():.5f} +- {se:.5f}")
    assert d.mean() < -2 * se
    assert r[:, 3].mean() > r[:, 1].mean()
