"""GPU parity of the plain path on the vector models (Lorenz 63, OU) against
the FP64 oracle, through the C ABI (MI355X only).

Every case feeds both sides identical inputs (seeded particle clouds,
log-weights and observations, and the same Philox counters) and compares
element by element: states and log-weights within 1e-5 relative, ancestors
identical outside the 1e-6 CDF band, estimators to FP64 accumulation
accuracy; the end-to-end test compares the MSE against the simulated truth
over 32 seeds within two standard errors of the oracle's.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import pf_inputs
from pf_testlib import (assert_rel_close, band_mask, oracle_to_vec, vec_to_oracle)

pytestmark = pytest.mark.gpu

L63 = pf_inputs.lorenz63()
OU = pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)


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


def _ctx(pf, spec, M, N, seed, fused=False):
    return pf.ParticleFilter([spec], [(0, M, N, seed)], fused=fused)


def _dev(torch, a, dtype=None):
    import torch as _t
    t = _t.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


# ------------------------------------------------------------------ RNG -------
@pytest.mark.parametrize("seed,c1,c2,c3,n", [(1, 0, 0, 2 << 24, 4099), (0xDEADBEEF12345678, 7, 123, (3 << 24) | 5, 1000),
                                          (5, 0xFFFFFFFF, 9, 6 << 24, 17)])
def test_philox_bits_and_normals(pf, orc, torch_mod, seed, c1, c2, c3, n):
    bits, z = pf.philox_stream(seed, c1, c2, c3, n)
    torch_mod.cuda.synchronize()
    ob = orc.philox_stream(seed, c1, c2, c3, n)
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), ob)
    oz = orc.normal_stream(seed, c1, c2, c3, n)
    assert_rel_close(z.cpu().numpy(), oz, floor=1.0, what="normals")


# ------------------------------------------------------------------ init ------
@pytest.mark.parametrize("spec,M,N", [(L63, 3, 1000), (OU, 2, 77)])
def test_prior_draw(pf, orc, torch_mod, spec, M, N):
    f = _ctx(pf, spec, M, N, seed=5)
    x = f.get_particles(0).cpu().numpy()
    m = orc.Model(spec)
    for k in range(M):
        ref = orc.init(m, 5, k, N)
        assert_rel_close(vec_to_oracle(x)[k], ref, floor=1.0, what="prior draw")


# ------------------------------------------------------------------ propagate -
@pytest.mark.parametrize("spec,M,N,t", [(L63, 4, 256, 1), (L63, 3, 1000, 7), (L63, 1, 1, 3),
                                        (OU, 2, 513, 2), (L63, 2, 300, 101)])
def test_propagate_and_weight(pf, orc, torch_mod, spec, M, N, t):
    seed = 1234 + N
    X0 = pf_inputs.particles(seed, spec, M, N, spread=3.0).astype(np.float32)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 99, 1)
    y32 = y[0].astype(np.float32)
    f = _ctx(pf, spec, M, N, seed=seed)
    f.set_particles(0, _dev(torch_mod, oracle_to_vec(X0)))
    f.set_interval(t)
    f.run_stages(pf.STAGE_PROPAGATE | pf.STAGE_WEIGHT, _dev(torch_mod, y32))
    xb = vec_to_oracle(f.get_predicted(0).cpu().numpy())
    lw = f.get_logweights(0).cpu().numpy()
    for k in range(M):
        ref = orc.propagate(m, seed, k, t, X0[k].astype(np.float64))
        assert_rel_close(xb[k], ref, floor=1.0, what="propagated states")
        rlw = orc.weights(m, ref, y32.astype(np.float64))
        assert_rel_close(lw[k], rlw, floor=1.0, what="log-weights")


# ------------------------------------------------------------------ resample --
def _check_resample(pf, orc, torch_mod, M, N, t, lw, seed):
    f = _ctx(pf, L63, M, N, seed=seed)
    f.set_logweights(0, _dev(torch_mod, lw))
    f.set_interval(t)
    f.run_stages(pf.STAGE_RESAMPLE)
    A = f.get_ancestors(0).cpu().numpy()
    st = f.get_filter_stats(0).cpu().numpy()
    n_diff = 0
    for k in range(M):
        lwk = lw[k].astype(np.float64)
        Ao, Co, Uo, (mx, W, s2, deg) = orc.resample(seed, k, t, lwk)
        band = band_mask(Co, Uo)
        assert np.all(np.diff(A[k]) >= 0), "ancestors not ascending"
        assert A[k].min() >= 0 and A[k].max() < N
        mism = (A[k] != Ao) & ~band
        assert not mism.any(), (k, np.argwhere(mism)[:5].ravel(), A[k][mism][:5], Ao[mism][:5])
        n_diff += int((A[k] != Ao).sum())
        assert st[k, 3] == float(deg)
        if not deg:
            assert st[k, 0] == mx
            assert st[k, 1] == pytest.approx(W, rel=1e-12)
            assert st[k, 2] == pytest.approx(s2, rel=1e-12)
    # At large N the CDF values are ~1/N apart, so most uniforms lie within
    # 1e-6 of one; both sides keep the CDF and the spacings in FP64, so the
    # ancestors must in fact agree almost everywhere, band or not.
    assert n_diff <= max(4, 1e-5 * M * N), n_diff
    return f, A


@pytest.mark.parametrize("M,N", [(1, 1), (2, 2), (3, 3), (2, 255), (1, 4095), (2, 4096), (3, 4097),
                                 (2, 8229), (1, 70001), (4, 256)])
def test_resample_matches_oracle(pf, orc, torch_mod, M, N):
    lw = pf_inputs.logweights(100 + N, M, N, scale=5.0)
    # a few impossible particles (NaN state -> -inf) and exact ties
    if N > 10:
        lw[:, 3] = -np.inf
        lw[:, 5] = lw[:, 4]
    _check_resample(pf, orc, torch_mod, M, N, t=17, lw=lw, seed=31 + N)


def test_resample_peaked_weights(pf, orc, torch_mod):
    # one dominant particle per filter (log-weights spread over hundreds)
    M, N = 3, 5000
    rng = np.random.default_rng(8)
    lw = (-200.0 * rng.random((M, N))).astype(np.float32)
    lw[np.arange(M), rng.integers(0, N, M)] = 0.0
    _check_resample(pf, orc, torch_mod, M, N, t=2, lw=lw, seed=77)


def test_resample_degenerate(pf, orc, torch_mod):
    M, N = 2, 300
    lw = np.full((M, N), -np.inf, dtype=np.float32)
    f, A = _check_resample(pf, orc, torch_mod, M, N, t=4, lw=lw, seed=3)
    _, _, logZ, _ = f.estimate()
    # degenerate weights: uniform resampling and log G = -inf
    f.run_stages(pf.STAGE_ESTIMATE)
    assert np.all(f.get_filter_stats(0).cpu().numpy()[:, 3] == 1.0)


def test_resample_full_size_one_filter(pf, orc, torch_mod):
    # the M = 1, N = 2^20 split of the Lorenz time-error sweep
    M, N = 1, 1 << 20
    lw = pf_inputs.logweights(5, M, N, scale=3.0)
    _check_resample(pf, orc, torch_mod, M, N, t=500, lw=lw, seed=2024)


# ------------------------------------------------------------------ gather / estimate
@pytest.mark.parametrize("M,N", [(4, 256), (2, 5000)])
def test_gather_and_estimators(pf, orc, torch_mod, M, N):
    seed = 555 + N
    Xb = pf_inputs.particles(seed, L63, M, N, spread=2.0).astype(np.float32)
    lw = pf_inputs.logweights(seed, M, N, scale=2.0)
    f = _ctx(pf, L63, M, N, seed=seed)
    f.set_predicted(0, _dev(torch_mod, oracle_to_vec(Xb)))
    f.set_logweights(0, _dev(torch_mod, lw))
    f.set_interval(9)
    f.run_stages(pf.STAGE_RESAMPLE | pf.STAGE_GATHER | pf.STAGE_ESTIMATE)
    A = f.get_ancestors(0).cpu().numpy()
    X = vec_to_oracle(f.get_particles(0).cpu().numpy())
    mean, mean_w, _, fmean = [t.cpu().numpy() for t in f.estimate()]
    fmean = fmean.reshape(M, 3)
    em = np.zeros(3)
    emw = np.zeros(3)
    for k in range(M):
        Ao, Co, Uo, (mx, W, s2, deg) = orc.resample(seed, k, 9, lw[k].astype(np.float64))
        assert np.array_equal(A[k][~band_mask(Co, Uo)], Ao[~band_mask(Co, Uo)])
        assert np.array_equal(X[k], Xb[k][A[k]])
        ref = orc.mean(Xb[k].astype(np.float64)[Ao])
        assert np.allclose(fmean[k], ref, rtol=1e-12, atol=1e-12)
        refw = orc.weighted_mean(Xb[k].astype(np.float64), lw[k].astype(np.float64), mx)
        em += ref / M
        emw += refw / M
    assert np.allclose(mean, em, rtol=1e-12, atol=1e-12)
    assert np.allclose(mean_w, emw, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ full step --
def test_first_interval_and_evidence(pf, orc, torch_mod):
    M, N, seed = 4, 256, 11
    m = orc.Model(L63)
    xt, y = orc.simulate(m, 40, 3)
    y32 = y.astype(np.float32)
    f = _ctx(pf, L63, M, N, seed=seed)
    f.step(_dev(torch_mod, y32[0]))
    _, _, logZ, _ = f.estimate()
    logZ = logZ.cpu().numpy()
    xb = vec_to_oracle(f.get_predicted(0).cpu().numpy())
    for k in range(M):
        X = orc.init(m, seed, k, N)
        r = orc.filter_interval(m, seed, k, 1, X, y32[0].astype(np.float64))
        ref = orc.propagate(m, seed, k, 1, orc.init(m, seed, k, N))
        assert_rel_close(xb[k], ref, what="interval-1 states")
        assert logZ[k] == pytest.approx(r["logZ"], rel=1e-5, abs=1e-5)


def test_determinism(pf, torch_mod):
    m_t = pf_inputs.lorenz63()
    outs = []
    for _ in range(2):
        f = _ctx(pf, m_t, 8, 3000, seed=9)
        y = torch_mod.tensor([1.0, 20.0], dtype=torch_mod.float32, device="cuda")
        for _t in range(5):
            f.step(y)
        outs.append([t.cpu().numpy() for t in f.estimate()])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def _oracle_mse(args):
    seed, T = args
    import oracle as orc
    m = orc.Model(pf_inputs.lorenz63())
    xt, y = orc.simulate(m, 10_000 + seed, T)
    y32 = y.astype(np.float32).astype(np.float64)
    est, _, _, _ = orc.run_ensemble(m, seed, 4, 256, y32)
    return float(np.mean((est - xt[1:]) ** 2))


def test_end_to_end_mse_32_seeds(pf, orc, torch_mod):
    # Lorenz 63, M = 4 filters x N = 256, T = 100 observations, seeds 1..32
    T = 100
    seeds = list(range(1, 33))
    m = orc.Model(L63)
    gpu = []
    for s in seeds:
        xt, y = orc.simulate(m, 10_000 + s, T)
        f = _ctx(pf, L63, 4, 256, seed=s)
        yd = _dev(torch_mod, y.astype(np.float32))
        est = np.zeros((T, 3))
        for t in range(T):
            f.step(yd[t])
            est[t] = f.estimate()[0].cpu().numpy()
        gpu.append(float(np.mean((est - xt[1:]) ** 2)))
    # the oracle's C calls release the GIL, so threads run the seeds in parallel
    with cf.ThreadPoolExecutor(8) as pool:
        ora = list(pool.map(_oracle_mse, [(s, T) for s in seeds]))
    gpu, ora = np.array(gpu), np.array(ora)
    se = ora.std(ddof=1) / np.sqrt(len(seeds))
    print(f"MSE gpu {gpu.mean():.5f} oracle {ora.mean():.5f} (2 SE = {2 * se:.5f}); "
          f"paired diff sd {np.std(gpu - ora, ddof=1) / np.sqrt(len(seeds)):.5f}")
    assert abs(gpu.mean() - ora.mean()) <= 2 * se
