"""GPU parity of the learned proposal (MI355X only).

* The BF16-MFMA MLP against the oracle's bfloat16-mode forward pass:
  bit-exact on dyadic parameters and inputs for which every FP32 partial sum
  is provably exact (so both sides take the same bfloat16 rounding
  decisions), and within the rounding bound on random values.
* A zero network reproduces the bootstrap FH-N interval: on the fused path
  states bit for bit and log-weights to FP32 summation-order rounding; on
  the plain path to the rounding of its per-launch compensated sums.
* A constant correction (only the output bias set): states and log-weights,
  density ratio included, against the oracle to the bootstrap tolerance
  (1e-5 relative, floor 0.1 for states and 1 for log-weights).
* Random networks: single intervals against the oracle with the tolerance
  that the bfloat16 rounding of the features implies (derived in the test).
"""
import numpy as np
import pytest

import pf_inputs
from pf_testlib import assert_rel_close

pytestmark = pytest.mark.gpu

F20 = pf_inputs.fhn(20)
F40 = pf_inputs.fhn(40)


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


def _dev(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _dyadic(orc, seed, in_dim, out_dim, rows):
    rng = np.random.default_rng(seed)
    p = np.zeros(orc.mlp_nparams(in_dim, out_dim))
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, in_dim, out_dim)
    W1[:] = rng.integers(-8, 9, W1.shape) / 16
    b1[:] = rng.integers(-8, 9, b1.shape) / 16
    W2[:] = rng.integers(-3, 4, W2.shape) / 16
    b2[:] = rng.integers(-8, 9, b2.shape) / 16
    W3[:] = rng.integers(-4, 5, W3.shape) / 16
    b3[:] = rng.integers(-8, 9, b3.shape) / 16
    X = rng.integers(-8, 9, (rows, in_dim)) / 8
    return p, X


def _granule(h):
    """Finest spacing among the positive bfloat16 values of each row."""
    pos = np.where(h > 0, h, 1.0)
    g = np.where(h > 0, 2.0 ** np.floor(np.log2(pos)) * 2.0 ** -7, np.inf)
    return g.min(1)


@pytest.mark.parametrize("in_dim,out_dim,rows", [(20, 2, 1000), (3, 1, 333), (20, 2, 16), (7, 4, 5)])
def test_mlp_forward_bit_exact_on_dyadic_values(pf, orc, torch_mod, in_dim, out_dim, rows):
    p, X = _dyadic(orc, in_dim + rows, in_dim, out_dim, rows)
    ref, h1, h2 = orc.mlp_forward(p, X, out_dim, bf16_mode=True)
    got = pf.mlp_forward(_dev(p), _dev(X), out_dim).cpu().numpy().astype(np.float64)
    # rows whose every partial sum is a multiple of a granule g with
    # sum |terms| < 2^24 g are exact in FP32 in any summation order
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, in_dim, out_dim)
    g2 = np.minimum(_granule(h1) / 16, 1 / 16)
    g3 = np.minimum(_granule(h2) / 16, 1 / 16)
    s2 = (np.abs(h1) @ np.abs(W2).T).max(1) + np.abs(b2).max()
    s3 = (np.abs(h2) @ np.abs(W3).T).max(1) + np.abs(b3).max()
    exact = (s2 / g2 < 2 ** 24) & (s3 / g3 < 2 ** 24)
    assert exact.mean() > 0.99
    assert np.array_equal(got[exact], ref[exact])
    assert np.all(np.abs(got - ref) <= 1e-2 * (1 + np.abs(ref)))


def test_mlp_forward_random_values(pf, orc, torch_mod):
    """Generic values: the two sides may round a hidden activation to
    neighbouring bfloat16 values when its FP32 and FP64 sums straddle a
    rounding boundary; an output then moves by at most sum_u |W3_u| ulp(h2_u)
    (plus the layer-1 flips seen through W2), which bounds the check."""
    rng = np.random.default_rng(5)
    in_dim, out_dim, rows = 20, 2, 4096
    p = rng.standard_normal(orc.mlp_nparams(in_dim, out_dim)) * 0.2
    X = rng.standard_normal((rows, in_dim)).astype(np.float32).astype(np.float64)
    ref, h1, h2 = orc.mlp_forward(p.astype(np.float32).astype(np.float64), X, out_dim,
                                  bf16_mode=True)
    got = pf.mlp_forward(_dev(p), _dev(X), out_dim).cpu().numpy().astype(np.float64)
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(orc.bf16(p.astype(np.float32)), in_dim, out_dim)
    bound = (np.abs(h2) @ np.abs(W3).T) * 2.0 ** -7 * 4 + 1e-5 * (1 + np.abs(ref))
    assert np.all(np.abs(got - ref) <= bound)
    close = np.abs(got - ref) <= 1e-5 * np.maximum(np.abs(ref), 0.1)
    assert close.mean() > 0.9, close.mean()


def _learned_filter(pf, spec, M, N, seed, fused, params=None):
    f = pf.ParticleFilter([spec], [(0, M, N, seed, pf.ENS_LEARNED)], fused=fused)
    if params is not None:
        f.set_proposal(0, _dev(params))
    return f


def _cloud(orc, spec, M, N, seed):
    m = orc.Model(spec)
    xt, _ = orc.simulate(m, 500 + seed, 10)
    rng = np.random.default_rng(seed)
    return (xt[-1] + 0.05 * rng.standard_normal((M, N, spec["dx"]))).astype(np.float32)


@pytest.mark.parametrize("fused", [False, True])
def test_zero_network_is_the_bootstrap_interval(pf, orc, torch_mod, fused):
    spec, M, N, seed, t = F20, 3, 40, 17, 4
    X0 = _cloud(orc, spec, M, N, seed)
    _, y = orc.simulate(orc.Model(spec), 801, t)
    yd = _dev(y[t - 1])
    out = []
    for learned in (False, True):
        ens = (0, M, N, seed, pf.ENS_LEARNED if learned else 0)
        f = pf.ParticleFilter([spec], [ens], fused=fused)
        f.set_particles(0, _dev(X0))
        f.set_interval(t)
        if fused:
            f.step(yd)
        else:
            f.run_stages(pf.STAGE_PROPAGATE | pf.STAGE_WEIGHT, yd)
        f.sync()
        out.append((f.get_predicted(0).cpu().numpy(), f.get_logweights(0).cpu().numpy()))
    if fused:
        # the same blocked stepping arithmetic with a zero correction
        assert np.array_equal(out[0][0], out[1][0])
        assert np.allclose(out[0][1], out[1][1], rtol=2e-6, atol=1e-6)
    else:
        # the plain bootstrap path streams one step per launch (its
        # compensated sums restart every step): rounding-level agreement
        assert_rel_close(out[1][0], out[0][0], floor=0.1, rel=1e-5, what="states")
        assert_rel_close(out[1][1], out[0][1], floor=1.0, rel=1e-5, what="log-weights")


# (an odd number of particles leaves the second particle slot of the last
# workgroup empty; J = 48 is the largest grid, whose LDS fills the CU)
@pytest.mark.parametrize("spec,M,N,fused", [(F20, 2, 5, False), (F20, 2, 4, True), (F40, 1, 2, True),
                                            (F20, 3, 3, True), (pf_inputs.fhn(48), 1, 3, True)])
def test_constant_correction_matches_oracle(pf, orc, torch_mod, spec, M, N, fused):
    seed, t = 31 + N, 3
    p = np.zeros(orc.mlp_nparams(22, 2))
    p[-2:] = [0.0625, -0.03125]  # b3: u_v, u_w (exact in bfloat16)
    X0 = _cloud(orc, spec, M, N, seed)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 802, t)
    y32 = y[t - 1].astype(np.float32)
    f = _learned_filter(pf, spec, M, N, seed, fused, p)
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
        Xr, dlw = orc.propagate_learned(m, p, seed, k, t, X0[k].astype(np.float64),
                                        y32.astype(np.float64))
        assert_rel_close(xb[k], Xr, floor=0.1, what="learned FH-N states")
        rlw = orc.weights(m, Xr, y32.astype(np.float64)) + dlw
        assert np.all(dlw < -1.0)  # the correction term is really there
        assert_rel_close(lw[k], rlw, floor=1.0, what="learned FH-N log-weights")


def test_random_network_interval_matches_oracle(pf, orc, torch_mod):
    """A feature whose FP32 and FP64 values round to different bfloat16
    numbers (about 1e-7 / 2^-9 of them) moves u by at most
    |W1| 2^-8 |feature| through the network; over S steps a state moves by
    at most h S of that, and the log-weight by the derivative of the ratio
    terms times it.  The test derives both bounds from the weights and
    requires the states of nearly every node to agree to 1e-5."""
    spec, M, N, seed, t = F20, 1, 4, 41, 2
    rng = np.random.default_rng(3)
    p = rng.standard_normal(orc.mlp_nparams(22, 2)) * 0.05
    p = p.astype(np.float32).astype(np.float64)
    X0 = _cloud(orc, spec, M, N, seed)
    m = orc.Model(spec)
    _, y = orc.simulate(m, 803, t)
    y32 = y[t - 1].astype(np.float32).astype(np.float64)
    f = _learned_filter(pf, spec, M, N, seed, True, p)
    f.set_particles(0, _dev(X0))
    f.set_interval(t)
    f.step(_dev(y32))
    f.sync()
    xb = f.get_predicted(0).cpu().numpy()[0].astype(np.float64)
    lw = f.get_logweights(0).cpu().numpy()[0].astype(np.float64)
    Xr, dlw = orc.propagate_learned(m, p, seed, 0, t, X0[0].astype(np.float64), y32)
    rlw = orc.weights(m, Xr, y32) + dlw
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(orc.bf16(p), 22, 2)
    lip = np.abs(W3).sum(1).max() * np.abs(W2).sum(1).max() * np.abs(W1).sum(1).max()
    du = lip * 2.0 ** -8 * 1.5       # one feature flip of a state of size <= 1.5
    dx_max = spec["h"] * spec["S"] * du * 4
    err = np.abs(xb - Xr)
    assert err.max() <= dx_max + 1e-5 * np.maximum(np.abs(Xr), 0.1).max(), (err.max(), dx_max)
    close = err <= 1e-5 * np.maximum(np.abs(Xr), 0.1)
    assert close.mean() > 0.99, close.mean()
    c = np.sqrt(spec["h"]) / spec["noise_sd"][0]
    dlw_max = 2 * spec["dx"] * spec["S"] * (c * 5.0 + 2 * c * c * 0.5) * du + 1e-4 * np.abs(rlw)
    assert np.all(np.abs(lw - rlw) <= dlw_max), (np.abs(lw - rlw).max(), dlw_max)
