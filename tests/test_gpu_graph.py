"""GPU tests of the graph-replayed fused interval (MI355X only).

Each interval after the first is one launch of a captured hipGraph that
reads the interval index and the observations from device memory.  Every
replay is compared with the eager fused path on the same seeds (identical
kernels and arguments, so bit-identical results are expected), with the
program's own eager work (estimate copies, synchronisations) between
replays, for the Lorenz model, the FH-N model, a mixed batch, the paper's
network with bootstrap and auxiliary ensembles, the other resampling schemes
with the ESS schedule, a learned-proposal ensemble, and a reset of the
interval counter in the middle of a run.
"""
import numpy as np
import pytest

import pf_inputs

pytestmark = pytest.mark.gpu


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


def _snap(f, n_ens):
    out = [t.cpu().numpy() for t in f.estimate()]
    for e in range(n_ens):
        out.append(f.get_ancestors(e).cpu().numpy())
        out.append(f.get_logweights(e).cpu().numpy())
    return out


def _compare_runs(pf, orc, torch_mod, specs, ens, T):
    models = [orc.Model(s) for s in specs]
    ys = []
    for e, en in enumerate(ens):
        _, y = orc.simulate(models[en[0]], 300 + e, T)
        ys.append(y.astype(np.float32))
    y_all = torch_mod.from_numpy(np.ascontiguousarray(np.concatenate(ys, axis=1))).cuda()
    eager = pf.ParticleFilter(specs, ens, fused=True)
    graph = pf.ParticleFilter(specs, ens, graph=True)
    graph.set_observations(y_all)
    for t in range(T):
        eager.step(y_all[t])
        graph.step()
        graph.sync()
        a, b = _snap(eager, len(ens)), _snap(graph, len(ens))
        for x, z in zip(a, b):
            assert np.array_equal(x, z, equal_nan=True), f"interval {t + 1} differs"
    return eager, graph, y_all


def test_graph_matches_eager_lorenz(pf, orc, torch_mod):
    _compare_runs(pf, orc, torch_mod, [pf_inputs.lorenz63()], [(0, 16, 700, 3)], T=9)


def test_graph_matches_eager_fhn(pf, orc, torch_mod):
    _compare_runs(pf, orc, torch_mod, [pf_inputs.fhn(20)], [(0, 3, 64, 5)], T=5)


def test_graph_matches_eager_mixed_batch(pf, orc, torch_mod):
    specs = [pf_inputs.lorenz63(), pf_inputs.fhn(20),
             pf_inputs.ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.3)]
    ens = [(0, 2, 3000, 1), (1, 2, 128, 2), (0, 5, 64, 3), (2, 4, 100, 4), (0, 1, 9000, 5)]
    _compare_runs(pf, orc, torch_mod, specs, ens, T=5)


def test_graph_matches_eager_network_and_auxiliary(pf, orc, torch_mod):
    # the paper's FH-N network (events drawn often), a bootstrap and an
    # auxiliary ensemble, several particles per workgroup
    spec = pf_inputs.fhn_paper(32, eps=0.3)
    ens = [(0, 2, 1500, 7), (0, 2, 700, 8, pf.ENS_AUXILIARY)]
    _compare_runs(pf, orc, torch_mod, [spec], ens, T=4)


def test_graph_matches_eager_schemes_and_schedule(pf, orc, torch_mod):
    # the other resampling schemes and the ESS-triggered schedule (the
    # per-filter resampler's second variant) beside a plain ensemble
    specs = [pf_inputs.lorenz63(), pf_inputs.fhn(20)]
    ens = [(0, 3, 2000, 1, 0, "systematic"), (0, 2, 700, 2, 0, "residual", 0.5),
           (0, 2, 4096, 3, 0, "stratified"), (1, 2, 64, 4, 0, "multinomial", 0.7),
           (0, 4, 300, 5)]
    _compare_runs(pf, orc, torch_mod, specs, ens, T=5)


def test_graph_matches_eager_learned_proposal(pf, orc, torch_mod):
    # a learned-proposal FH-N ensemble (random network) beside a bootstrap one
    spec = pf_inputs.fhn(20)
    T = 3
    _, y = orc.simulate(orc.Model(spec), 301, T)
    y2 = np.concatenate([y, y], axis=1).astype(np.float32)
    y_all = torch_mod.from_numpy(np.ascontiguousarray(y2)).cuda()
    rng = np.random.default_rng(11)
    params = torch_mod.from_numpy(
        (rng.standard_normal(orc.mlp_nparams(22, 2)) * 0.05).astype(np.float32)).cuda()
    ens = [(0, 2, 96, 6, pf.ENS_LEARNED), (0, 2, 64, 7)]
    eager = pf.ParticleFilter([spec], ens, fused=True)
    graph = pf.ParticleFilter([spec], ens, graph=True)
    for f in (eager, graph):
        f.set_proposal(0, params)
    graph.set_observations(y_all)
    for t in range(T):
        eager.step(y_all[t])
        graph.step()
        graph.sync()
        for x, z in zip(_snap(eager, 2), _snap(graph, 2)):
            assert np.array_equal(x, z, equal_nan=True), f"interval {t + 1} differs"


def test_graph_interval_reset(pf, orc, torch_mod):
    spec = pf_inputs.lorenz63()
    m = orc.Model(spec)
    _, y = orc.simulate(m, 9, 8)
    y_all = torch_mod.from_numpy(y.astype(np.float32)).cuda()
    eager = pf.ParticleFilter([spec], [(0, 4, 256, 7)], fused=True)
    graph = pf.ParticleFilter([spec], [(0, 4, 256, 7)], graph=True)
    graph.set_observations(y_all)
    for t in (1, 2, 3, 2, 3, 4):
        eager.set_interval(t)
        graph.set_interval(t)
        eager.step(y_all[t - 1])
        graph.step()
        graph.sync()
        for x, z in zip(_snap(eager, 1), _snap(graph, 1)):
            assert np.array_equal(x, z, equal_nan=True)
    assert graph.interval() == 5


def test_graph_rejects_running_past_the_record(pf, orc, torch_mod):
    spec = pf_inputs.lorenz63()
    y_all = torch_mod.zeros((2, 2), dtype=torch_mod.float32, device="cuda")
    f = pf.ParticleFilter([spec], [(0, 2, 64, 1)], graph=True)
    f.set_observations(y_all)
    f.step()
    f.step()
    with pytest.raises(pf.PFError):
        f.step()
