"""GPU parity at the full sizes of the FH-N workloads (MI355X only).

The FH-N 40 x 40 ensemble of 64 filters x 512 particles and the learned
ensemble of 64 x 128 run in the launch configurations the benchmark times:
every stepping kernel loops over many particles per workgroup there (the
blocked kernel's particle groups, the streaming kernel's two register sets
that hold the next two particles while it steps the current one in place, the
learned kernel's particle loop), which small parity cases never reach.  A sample of particles
spread over the whole index range -- the last ones included -- is checked
against the oracle, which propagates each particle on its own from the
particles the GPU holds:
  - prior draws and the interval-1 states and log-weights (1e-5 relative,
    floors 0.1 for states and 1 for log-weights);
  - per-filter resampling of interval 1 on the GPU's log-weights (ancestors
    equal outside the 1e-6 CDF band);
  - interval 2, whose propagation reads the interval-1 particles through the
    ancestors (fused) or through the gather kernel (plain).
"""
import concurrent.futures as cf

import numpy as np
import pytest

import pf_inputs
from pf_testlib import assert_rel_close, band_mask

pytestmark = pytest.mark.gpu

F40 = pf_inputs.fhn(40)
POOL = 16


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


def _sample(M, N, n, seed):
    """(filter, particle) pairs: random over the whole range plus the first
    and last particles and the last filter."""
    rng = np.random.default_rng(seed)
    flat = set(rng.choice(M * N, size=n - 4, replace=False).tolist())
    flat |= {0, N - 1, M * N - N, M * N - 1}
    flat = np.array(sorted(flat))
    return flat // N, flat % N


def _rows(x, fil, idx):
    """Sampled particles [n, dx] of a device tensor [M, N, dx] (grid layout)."""
    import torch
    fi = torch.from_numpy(fil).cuda()
    ii = torch.from_numpy(idx).cuda()
    return x[fi, ii].cpu().numpy().astype(np.float64)


def _check_resampling(orc, A, lw, seed, t, filters):
    n_diff = tot = 0
    for fm in filters:
        Ao, Co, Uo, _ = orc.resample(seed, int(fm), t, lw[fm].astype(np.float64))
        band = band_mask(Co, Uo)
        assert not ((A[fm] != Ao) & ~band).any(), f"filter {fm}: ancestors differ outside the band"
        n_diff += int((A[fm] != Ao).sum())
        tot += A[fm].size
    assert n_diff <= max(4, 1e-5 * tot), n_diff


def _propagate_rows(orc, m, seed, fil, idx, t, X_in):
    def one(k):
        return orc.propagate_particle(m, seed, int(fil[k]), int(idx[k]), t, X_in[k])
    with cf.ThreadPoolExecutor(POOL) as pool:
        return np.array(list(pool.map(one, range(len(fil)))))


def _two_intervals(pf, orc, torch_mod, fused, M=64, N=512, n_sample=96):
    spec, seed = F40, 1
    m = orc.Model(spec)
    _, y = orc.simulate(m, 61, 2)
    y32 = y.astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=fused)
    fil, idx = _sample(M, N, n_sample, 5)
    print(f"FH-N 40x40 {M}x{N} {'fused' if fused else 'plain'}: {len(fil)} sampled particles",
          flush=True)
    x0 = _rows(f.get_particles(0), fil, idx)
    ref0 = np.array([orc.prior_particle(m, seed, int(a), int(b)) for a, b in zip(fil, idx)])
    assert_rel_close(x0, ref0, floor=0.1, what="prior draws")
    f.step(_dev(y32[0]))
    f.sync()
    xb1 = f.get_predicted(0)
    lw1 = f.get_logweights(0).cpu().numpy()
    A1 = f.get_ancestors(0).cpu().numpy()
    ref1 = _propagate_rows(orc, m, seed, fil, idx, 1, x0)
    assert_rel_close(_rows(xb1, fil, idx), ref1, floor=0.1, what="interval-1 states")
    rlw1 = np.array([orc.loglik(m, r, y32[0].astype(np.float64)) for r in ref1])
    assert_rel_close(lw1[fil, idx], rlw1, floor=1.0, what="interval-1 log-weights")
    _check_resampling(orc, A1, lw1, seed, 1, sorted(set(fil.tolist()) | {0, M - 1}))
    # interval 2 starts from the interval-1 particles the ancestors select
    x_in = _rows(xb1, fil, A1[fil, idx])
    del xb1
    if fused:
        f.step(_dev(y32[1]))
    else:
        f.run_stages(pf.STAGE_PROPAGATE | pf.STAGE_WEIGHT, _dev(y32[1]))
    f.sync()
    ref2 = _propagate_rows(orc, m, seed, fil, idx, 2, x_in)
    assert_rel_close(_rows(f.get_predicted(0), fil, idx), ref2, floor=0.1,
                     what="interval-2 states")
    lw2 = f.get_logweights(0).cpu().numpy()
    rlw2 = np.array([orc.loglik(m, r, y32[1].astype(np.float64)) for r in ref2])
    assert_rel_close(lw2[fil, idx], rlw2, floor=1.0, what="interval-2 log-weights")
    if fused:
        _check_resampling(orc, f.get_ancestors(0).cpu().numpy(), lw2, seed, 2,
                          sorted(set(fil.tolist()))[:16])


def test_fhn40_64x512_fused_two_intervals(pf, orc, torch_mod):
    """The blocked stepping kernel (all 20 Euler steps with the plane in LDS)
    over its particle groups, the second interval gathering through the
    pending ancestors."""
    _two_intervals(pf, orc, torch_mod, fused=True)


def test_fhn40_64x512_plain_stream_steps(pf, orc, torch_mod):
    """The streaming one-step kernel, 20 launches per interval: each
    workgroup has particles p + gridDim and p + 2 gridDim in flight while it
    steps p in place (32768 particles over 768 workgroups: both register sets,
    and workgroups with an odd and with an even particle count); the second
    interval reads the particles the gather kernel wrote."""
    _two_intervals(pf, orc, torch_mod, fused=False)


def test_fhn40_plain_stream_steps_between_one_and_two_rounds(pf, orc, torch_mod):
    """The streaming kernel where the particles number between one and two
    per resident workgroup (2 x 500 = 1000 particles over 768 workgroups on
    the MI355X): the first workgroups step a second particle from their
    second register set, the others stop after one."""
    _two_intervals(pf, orc, torch_mod, fused=False, M=2, N=500, n_sample=48)


def _learned_interval(pf, orc, torch_mod, p, n_sample, seed_sample):
    spec, M, N, seed = F40, 64, 128, 2
    m = orc.Model(spec)
    _, y = orc.simulate(m, 62, 1)
    y32 = y[0].astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed, pf.ENS_LEARNED)], fused=True)
    f.set_proposal(0, _dev(p.astype(np.float32)))
    fil, idx = _sample(M, N, n_sample, seed_sample)
    print(f"learned FH-N 40x40 {M}x{N}: {len(fil)} sampled particles", flush=True)
    x0 = _rows(f.get_particles(0), fil, idx)
    f.step(_dev(y32))
    f.sync()
    xb = _rows(f.get_predicted(0), fil, idx)
    lw = f.get_logweights(0).cpu().numpy()
    A = f.get_ancestors(0).cpu().numpy()
    yd = y32.astype(np.float64)

    def one(k):
        return orc.propagate_learned_particle(m, p, seed, int(fil[k]), int(idx[k]), 1, x0[k], yd)
    with cf.ThreadPoolExecutor(POOL) as pool:
        res = list(pool.map(one, range(len(fil))))
    ref = np.array([r[0] for r in res])
    rlw = np.array([orc.loglik(m, r[0], yd) + r[1] for r in res])
    _check_resampling(orc, A, lw, seed, 1, sorted(set(fil.tolist()))[:16])
    return spec, xb, ref, lw[fil, idx], rlw, np.array([r[1] for r in res])


def test_learned_64x128_constant_correction(pf, orc, torch_mod):
    """Only the output bias set (exact in bfloat16): every tile of the MLP
    runs, the correction is a known constant, and states and log-weights
    (density ratio included) meet the bootstrap tolerance."""
    p = np.zeros(orc.mlp_nparams(22, 2))
    p[-2:] = [0.0625, -0.03125]
    spec, xb, ref, lw, rlw, dlw = _learned_interval(pf, orc, torch_mod, p, 48, 11)
    assert np.all(dlw < -1.0)
    assert_rel_close(xb, ref, floor=0.1, what="learned states")
    assert_rel_close(lw, rlw, floor=1.0, what="learned log-weights")


def test_learned_64x128_random_network(pf, orc, torch_mod):
    """A random network: a feature whose FP32 and FP64 values round to
    different bfloat16 numbers moves u by at most the network's Lipschitz
    constant times one bfloat16 unit; the states of nearly every node agree
    to 1e-5 and all within the bound that this implies."""
    rng = np.random.default_rng(4)
    p = (rng.standard_normal(orc.mlp_nparams(22, 2)) * 0.05).astype(np.float32).astype(np.float64)
    spec, xb, ref, lw, rlw, _ = _learned_interval(pf, orc, torch_mod, p, 32, 12)
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(orc.bf16(p), 22, 2)
    lip = np.abs(W3).sum(1).max() * np.abs(W2).sum(1).max() * np.abs(W1).sum(1).max()
    du = lip * 2.0 ** -8 * 1.5
    dx_max = spec["h"] * spec["S"] * du * 4
    err = np.abs(xb - ref)
    assert err.max() <= dx_max + 1e-5 * np.maximum(np.abs(ref), 0.1).max(), (err.max(), dx_max)
    close = err <= 1e-5 * np.maximum(np.abs(ref), 0.1)
    assert close.mean() > 0.99, close.mean()
    c = np.sqrt(spec["h"]) / spec["noise_sd"][0]
    dlw_max = 2 * spec["dx"] * spec["S"] * (c * 5.0 + 2 * c * c * 0.5) * du + 1e-4 * np.abs(rlw)
    assert np.all(np.abs(lw - rlw) <= dlw_max), (np.abs(lw - rlw).max(), dlw_max)
