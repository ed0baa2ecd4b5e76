"""GPU parity of the auxiliary particle filter ensembles (PF_ENS_AUXILIARY)
against the FP64 oracle's auxiliary filter, through the C ABI (MI355X only).

From identical particles and carried log-weights (seeded), one interval on
both sides: the pilot, the first-stage ancestors (the slots whose first-stage
ancestor differs -- a uniform within the CDF band, where the FP32 and FP64
pilot weights can fall on either side -- are counted and bounded), the
propagated states and second-stage log-weights within 1e-5 relative, the
carried log-weights, the weighted estimate and log G.  Two intervals from the
prior draw on both sides for the FH-N grid; and auxiliary ensembles in a
mixed batch equal themselves run alone, bit for bit.
"""
import numpy as np
import pytest

import pf_inputs
from pf_testlib import oracle_to_vec, rel_close, vec_to_oracle

pytestmark = pytest.mark.gpu

L63 = pf_inputs.lorenz63()
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
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _carried(seed, M, N, spread):
    rng = np.random.default_rng(seed)
    w = np.exp(spread * rng.standard_normal((M, N)))
    return np.log(N * w / w.sum(axis=1, keepdims=True))


def _check(k, xg, lwg, lwcg, xo, r, floor, min_frac=0.99):
    """Slots whose state and log-weight agree within 1e-5 (they share their
    first-stage ancestor); at least min_frac of them."""
    okx = rel_close(xg, xo, floor=floor).all(axis=1)
    okl = rel_close(lwg, r["lw"], floor=1.0)
    ok = okx & okl
    assert ok.mean() >= min_frac, (k, ok.mean())
    assert rel_close(lwcg[ok], r["lwc"][ok], floor=1.0).all(), k
    return ok


@pytest.mark.parametrize("scheme", ["multinomial", "systematic", "residual"])
def test_apf_interval_matches_oracle_lorenz(pf, orc, torch_mod, scheme):
    M, N, seed, t = 4, 512, 4321, 2
    print(f"APF Lorenz {scheme}", flush=True)
    m = orc.Model(L63)
    _, y = orc.simulate(m, 66, t)
    y32 = y[t - 1].astype(np.float32)
    X0 = pf_inputs.particles(seed, L63, M, N, spread=1.5).astype(np.float32)
    lwc0 = _carried(seed, M, N, 0.7).astype(np.float32)
    f = pf.ParticleFilter([L63], [(0, M, N, seed, pf.ENS_AUXILIARY, scheme, 0.0)], fused=True)
    f.set_particles(0, _dev(oracle_to_vec(X0)))
    f.set_carried_logweights(0, _dev(lwc0))
    f.set_interval(t)
    f.step(_dev(y32))
    xb = vec_to_oracle(f.get_predicted(0).cpu().numpy())
    lw = f.get_logweights(0).cpu().numpy()
    lwc = f.get_carried_logweights(0).cpu().numpy()
    A = f.get_ancestors(0).cpu().numpy()
    _, _, logZ, fmean = [v.cpu().numpy() for v in f.estimate()]
    fmean = fmean.reshape(M, 3)
    f.close()
    for k in range(M):
        r = orc.apf_interval(m, seed, k, t, X0[k].astype(np.float64), lwc0[k].astype(np.float64),
                             y32.astype(np.float64), 0.0, scheme)
        ok = _check(k, xb[k], lw[k], lwc[k], r["X"], r, floor=1.0)
        # the interval ends without resampling: identity ancestors
        assert np.array_equal(A[k], np.arange(N))
        if ok.all():
            assert logZ[k] == pytest.approx(r["logZ"], rel=1e-5, abs=1e-4)
            assert rel_close(fmean[k], r["mean_w"], floor=1.0).all(), k


def test_apf_two_intervals_fhn_grid(pf, orc, torch_mod):
    # FH-N 20 x 20, 2 filters of 128, intervals 1 and 2 from the prior draw
    M, N, seed, T = 2, 128, 808, 2
    print("APF FH-N 20x20", flush=True)
    m = orc.Model(F20)
    _, y = orc.simulate(m, 9, T)
    y32 = y.astype(np.float32)
    f = pf.ParticleFilter([F20], [(0, M, N, seed, pf.ENS_AUXILIARY, "stratified", 0.0)],
                          fused=True)
    for t in range(T):
        f.step(_dev(y32[t]))
    xb = f.get_predicted(0).cpu().numpy()
    lw = f.get_logweights(0).cpu().numpy()
    lwc = f.get_carried_logweights(0).cpu().numpy()
    f.close()
    for k in range(M):
        X = orc.init(m, seed, k, N)
        lwck = np.zeros(N)
        for t in range(1, T + 1):
            r = orc.apf_interval(m, seed, k, t, X, lwck, y32[t - 1].astype(np.float64), 0.0,
                                 "stratified")
            X, lwck = r["X"], r["lwc"]
        _check(k, xb[k], lw[k], lwc[k], r["X"], r, floor=0.1, min_frac=0.98)


def test_apf_batch_members_equal_runs_alone(pf, torch_mod):
    ens = [(0, 2, 300, 21, pf.ENS_AUXILIARY), (0, 3, 256, 22),
           (1, 2, 128, 23, pf.ENS_AUXILIARY, "residual", 0.0), (0, 1, 900, 24, 0, "systematic", 0.7),
           (0, 2, 1000, 25, pf.ENS_AUXILIARY, "stratified", 0.0)]
    specs = [L63, F20]
    T = 3
    sim = pf.ParticleFilter(specs, [(0, 1, 1, 1), (1, 1, 1, 1)], fused=True)
    ys = [sim.simulate(e[0], 50 + i, T)[1] for i, e in enumerate(ens)]
    sim.close()
    y_all = torch_mod.cat(ys, dim=1).contiguous()
    for graph in (False, True):
        print(f"APF batch graph={graph}", flush=True)
        f = pf.ParticleFilter(specs, ens, fused=True, graph=graph)
        if graph:
            f.set_observations(y_all)
        for t in range(T):
            f.step(None if graph else y_all[t])
        batch = [(f.get_predicted(e).cpu().numpy(), f.get_logweights(e).cpu().numpy())
                 for e in range(len(ens))]
        lz = f.estimate()[2].cpu().numpy()
        f.close()
        off = 0
        for e, d in enumerate(ens):
            g = pf.ParticleFilter([specs[d[0]]], [(0,) + tuple(d[1:])], fused=True)
            for t in range(T):
                g.step(ys[e][t].contiguous())
            assert np.array_equal(batch[e][0], g.get_predicted(0).cpu().numpy()), e
            assert np.array_equal(batch[e][1], g.get_logweights(0).cpu().numpy()), e
            assert np.array_equal(lz[off:off + d[1]], g.estimate()[2].cpu().numpy()), e
            off += d[1]
            g.close()
