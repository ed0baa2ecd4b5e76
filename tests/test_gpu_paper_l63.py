"""The paper's own Lorenz 63 experiment (Sec. 4.1-4.2: x1 observed every 100
Euler steps with variance 1/2, unit diffusion, prior N(x*, 10 I)) on the GPU
against the FP64 oracle (MI355X only): for the ensemble of M = 20 filters of
N = 100 particles and for the centralised filter of K = M N = 2000, the MSE
of the estimate against the simulated truth over 32 seeds lies within two
standard errors of the oracle's (both sides run the same algorithm on their
own arithmetic, from the same Philox counters); and the batched run of many
independent ensembles on one graph-replayed context equals each ensemble
run alone."""
import concurrent.futures as cf

import numpy as np
import pytest

import pf_inputs

pytestmark = pytest.mark.gpu

SPEC = pf_inputs.lorenz63_paper()
T = 10


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


def _oracle_mse(args):
    seed, M, N = args
    import oracle as orc
    m = orc.Model(SPEC)
    xt, y = orc.simulate(m, 20_000 + seed, T)
    y32 = y.astype(np.float32).astype(np.float64)
    est, _, _, _ = orc.run_ensemble(m, seed, M, N, y32)
    return float(np.mean((est - xt[1:]) ** 2))


@pytest.mark.parametrize("M,N", [(20, 100), (1, 2000)])
def test_paper_lorenz_mse_matches_oracle_32_seeds(pf, orc, torch_mod, M, N):
    torch = torch_mod
    seeds = list(range(1, 33))
    m = orc.Model(SPEC)
    gpu = []
    for s in seeds:
        print(f"paper Lorenz M {M} N {N} seed {s}", flush=True)
        xt, y = orc.simulate(m, 20_000 + s, T)
        f = pf.ParticleFilter([SPEC], [(0, M, N, s)], fused=True)
        yd = torch.from_numpy(y.astype(np.float32)).cuda()
        est = np.zeros((T, 3))
        for t in range(T):
            f.step(yd[t])
            est[t] = f.estimate()[0].cpu().numpy()
        f.close()
        gpu.append(float(np.mean((est - xt[1:]) ** 2)))
    with cf.ThreadPoolExecutor(8) as pool:
        ora = list(pool.map(_oracle_mse, [(s, M, N) for s in seeds]))
    gpu, ora = np.array(gpu), np.array(ora)
    se = ora.std(ddof=1) / np.sqrt(len(seeds))
    print(f"MSE gpu {gpu.mean():.5f} oracle {ora.mean():.5f} (2 SE = {2 * se:.5f})")
    assert abs(gpu.mean() - ora.mean()) <= 2 * se


def test_batched_runs_equal_runs_alone(pf, torch_mod):
    # 8 runs of the M = 20 x N = 100 ensemble (and of the K = 2000 and
    # K = 20000 centralised filters) batched in one graph-replayed context:
    # each estimate at t = T equals that run alone (filters are independent,
    # Definition 3)
    torch = torch_mod
    orc_y = None
    sim = pf.ParticleFilter([SPEC], [(0, 1, 1, 1)], fused=True)
    _, y = sim.simulate(0, 3, T)
    sim.close()
    del orc_y
    for M, N in ((20, 100), (1, 2000), (1, 20000)):
        print(f"batched paper Lorenz M {M} N {N}", flush=True)
        ens = [(0, M, N, 700 + i) for i in range(8)]
        f = pf.ParticleFilter([SPEC], ens, graph=True)
        f.set_observations(y.repeat(1, len(ens)).contiguous())
        for _ in range(T):
            f.step()
        batch = f.estimate()[0].view(len(ens), 3).cpu().numpy()
        f.close()
        for i, e in enumerate(ens):
            g = pf.ParticleFilter([SPEC], [e], graph=True)
            g.set_observations(y.contiguous())
            for _ in range(T):
                g.step()
            alone = g.estimate()[0].cpu().numpy()
            g.close()
            assert np.array_equal(batch[i], alone), (M, N, i, batch[i], alone)
