"""GPU parity of the FitzHugh-Nagumo grid model against the FP64 oracle
(MI355X only): prior draw, the streaming one-step kernel (plain path) and the
temporally-blocked kernel (fused path) with the log-weights, per-filter
resampling on identical log-weights, the post-resampling and weighted
estimators, plain against fused, and the MSE against the simulated truth over
32 seeds on the reduced 20 x 20 workload.  States within 1e-5 relative with a
floor of 0.1 (the resting v and w are near 0), log-weights within 1e-5
relative with a floor of 1.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import pf_inputs
from pf_testlib import assert_rel_close, band_mask

pytestmark = pytest.mark.gpu

F20 = pf_inputs.fhn(20)
F40 = pf_inputs.fhn(40)
# grid sides that are not multiples of 4 (a slot of 4 nodes may straddle two
# rows: the stepping kernel's general neighbour path) and a small one that is
F10 = pf_inputs.fhn(10)
F12 = pf_inputs.fhn(12)
F42 = pf_inputs.fhn(42)


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
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _cloud(spec, M, N, seed):
    """A particle cloud around a travelling wave: the truth at t = 10, jittered."""
    import oracle as orc
    m = orc.Model(spec)
    xt, _ = orc.simulate(m, 500 + seed, 10)
    rng = np.random.default_rng(seed)
    X = xt[-1] + 0.05 * rng.standard_normal((M, N, spec["dx"]))
    return X.astype(np.float32)


@pytest.mark.parametrize("spec,M,N", [(F20, 2, 37), (F40, 1, 5)])
def test_prior_draw(pf, orc, torch_mod, spec, M, N):
    f = pf.ParticleFilter([spec], [(0, M, N, 9)])
    x = f.get_particles(0).cpu().numpy()
    m = orc.Model(spec)
    for k in range(M):
        assert_rel_close(x[k], orc.init(m, 9, k, N), floor=0.1, what="prior draw")


@pytest.mark.parametrize("spec,M,N,t,fused", [(F20, 2, 16, 3, False), (F20, 3, 7, 1, True),
                                              (F40, 1, 6, 2, False), (F40, 2, 4, 5, True),
                                              (F10, 2, 5, 2, True), (F12, 2, 4, 2, True),
                                              (F42, 1, 3, 1, True), (F10, 2, 3, 2, False)])
def test_propagate_and_weight(pf, orc, torch_mod, spec, M, N, t, fused):
    seed = 70 + N
    X0 = _cloud(spec, M, N, seed)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 800, t)
    y32 = y[t - 1].astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=fused)
    f.set_particles(0, _dev(X0))
    f.set_interval(t)
    if fused:
        f.step(_dev(y32))
    else:
        f.run_stages(pf.STAGE_PROPAGATE | pf.STAGE_WEIGHT, _dev(y32))
    f.sync()
    xb = f.get_predicted(0).cpu().numpy()
    lw = f.get_logweights(0).cpu().numpy()
    for k in range(M):
        ref = orc.propagate(m, seed, k, t, X0[k].astype(np.float64))
        assert_rel_close(xb[k], ref, floor=0.1, what="FH-N states")
        rlw = orc.weights(m, ref, y32.astype(np.float64))
        assert_rel_close(lw[k], rlw, floor=1.0, what="FH-N log-weights")


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("M,N", [(3, 64), (2, 513), (1, 4097)])
def test_resampling_and_estimators(pf, orc, torch_mod, M, N, fused):
    spec = F20
    seed, t = 5 + N, 11
    Xb = _cloud(spec, M, N, seed)
    lw = pf_inputs.logweights(seed, M, N, scale=6.0)
    lw[:, 1] = -np.inf
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=fused)
    f.set_predicted(0, _dev(Xb))
    f.set_logweights(0, _dev(lw))
    f.set_interval(t)
    f.run_stages(pf.STAGE_RESAMPLE | pf.STAGE_ESTIMATE if not fused else pf.STAGE_RESAMPLE)
    f.sync()
    A = f.get_ancestors(0).cpu().numpy()
    mean, mean_w, _, fmean = [x.cpu().numpy() for x in f.estimate()]
    fmean = fmean.reshape(M, spec["dx"])
    em = np.zeros(spec["dx"])
    emw = np.zeros(spec["dx"])
    n_diff = 0
    for k in range(M):
        Ao, Co, Uo, (mx, W, s2, deg) = orc.resample(seed, k, t, lw[k].astype(np.float64))
        band = band_mask(Co, Uo)
        assert not ((A[k] != Ao) & ~band).any()
        n_diff += int((A[k] != Ao).sum())
        ref = orc.mean(Xb[k].astype(np.float64)[A[k]])
        assert np.allclose(fmean[k], ref, rtol=1e-10, atol=1e-10)
        refw = orc.weighted_mean(Xb[k].astype(np.float64), lw[k].astype(np.float64), mx)
        em += ref / M
        emw += refw / M
    assert n_diff <= max(4, 1e-5 * M * N)
    assert np.allclose(mean, em, rtol=1e-10, atol=1e-10)
    assert np.allclose(mean_w, emw, rtol=1e-9, atol=1e-10)


def test_gather_hook_and_pending(pf, orc, torch_mod):
    spec, M, N = F20, 2, 50
    m = orc.Model(spec)
    _, y = orc.simulate(m, 3, 2)
    f = pf.ParticleFilter([spec], [(0, M, N, 4)], fused=True)
    f.step(_dev(y[0].astype(np.float32)))
    f.sync()
    xb = f.get_predicted(0).cpu().numpy()
    A = f.get_ancestors(0).cpu().numpy()
    x = f.get_particles(0).cpu().numpy()  # gathered through the pending ancestors
    for k in range(M):
        assert np.array_equal(x[k], xb[k][A[k]])


def test_plain_matches_fused(pf, orc, torch_mod):
    spec, M, N = F20, 3, 96
    m = orc.Model(spec)
    _, y = orc.simulate(m, 12, 3)
    yd = _dev(y.astype(np.float32))
    fp = pf.ParticleFilter([spec], [(0, M, N, 21)], fused=False)
    ff = pf.ParticleFilter([spec], [(0, M, N, 21)], fused=True)
    fp.step(yd[0])
    ff.step(yd[0])
    ff.sync()
    assert_rel_close(ff.get_predicted(0).cpu().numpy(), fp.get_predicted(0).cpu().numpy(),
                     floor=0.1, rel=1e-5, what="fused vs plain FH-N states")
    assert_rel_close(ff.get_logweights(0).cpu().numpy(), fp.get_logweights(0).cpu().numpy(),
                     floor=1.0, rel=1e-5, what="fused vs plain FH-N log-weights")


def _oracle_mse(args):
    seed, T = args
    import oracle as orc
    m = orc.Model(pf_inputs.fhn(20))
    xt, y = orc.simulate(m, 40_000 + seed, T)
    est, _, _, _ = orc.run_ensemble(m, seed, 4, 64, y.astype(np.float32).astype(np.float64))
    return float(np.mean((est[:, :400] - xt[1:, :400]) ** 2))


def test_end_to_end_mse_32_seeds(pf, orc, torch_mod):
    # FH-N 20 x 20, M = 4 x N = 64, T = 20, seeds 1..32 (fused path)
    T = 20
    seeds = list(range(1, 33))
    m = orc.Model(F20)
    gpu = []
    for s in seeds:
        xt, y = orc.simulate(m, 40_000 + s, T)
        f = pf.ParticleFilter([F20], [(0, 4, 64, s)], fused=True)
        yd = _dev(y.astype(np.float32))
        est = np.zeros((T, 800))
        for t in range(T):
            f.step(yd[t])
            est[t] = f.estimate()[0].cpu().numpy()
        f.sync()
        gpu.append(float(np.mean((est[:, :400] - xt[1:, :400]) ** 2)))
    with cf.ThreadPoolExecutor(16) as pool:
        ora = list(pool.map(_oracle_mse, [(s, T) for s in seeds]))
    gpu, ora = np.array(gpu), np.array(ora)
    se = ora.std(ddof=1) / np.sqrt(len(seeds))
    print(f"FH-N MSE(v) gpu {gpu.mean():.5f} oracle {ora.mean():.5f} (2 SE = {2 * se:.5f})")
    assert abs(gpu.mean() - ora.mean()) <= 2 * se
