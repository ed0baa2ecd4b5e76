"""GPU parity of the paper's modified FH-N network (PF_MODEL_FHN_PAPER: Sec.
5.1, 5.2) against the FP64 oracle, through the C ABI (MI355X only).

Identical inputs on both sides (seeded particle clouds at rest with a few
nodes inside the stimulus band, seeded event rings, the same Philox
counters): U and V within
1e-5 relative (floor 0.1), the event rings exactly, log-weights within 1e-5
(floor 1), on the plain and the fused path, one and several Euler steps per
interval, with a high event rate so that stimuli do happen.  Whether a node
lies in the open band (u-, u+) is a decision each side takes in its own
precision: a particle whose U comes within 2e-5 of a threshold at the start
of a step after the first is exempt (counted; at most 5%).  Also the prior draw,
the truth simulator, the 32-seed MSE against the oracle's, and a mixed batch
whose members equal themselves run alone.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import pf_inputs
from pf_testlib import assert_rel_close

pytestmark = pytest.mark.gpu

J = 32
NN = J * J


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


def _cloud(seed, spec, M, N, nn=NN, empty_rings=False):
    """Particles near the rest point with 8 nodes each in the middle of the
    stimulus band (so that the region is never empty), and random event
    rings (or rings without events)."""
    rng = np.random.default_rng(seed)
    dx = spec["dx"]
    X = np.full((M, N, dx), -1.0)
    X[:, :, :nn] = -1.03 + 0.05 * rng.standard_normal((M, N, nn))
    for k in range(M):
        for i in range(N):
            X[k, i, rng.choice(nn, 8, replace=False)] = -1.7 + 0.02 * rng.standard_normal(8)
    X[:, :, nn:2 * nn] = -2.6 + 0.1 * rng.standard_normal((M, N, nn))
    ring = rng.integers(-1, nn, size=(M, N, 25))
    ring[rng.random((M, N, 25)) < 0.6] = -1
    if empty_rings:
        ring[:] = -1
    X[:, :, 2 * nn:2 * nn + 25] = ring
    return X.astype(np.float32).astype(np.float64)


def _near_band(U, lo=-1.8, hi=-1.6, tol=2e-5):
    return np.any(np.abs(U - lo) < tol) or np.any(np.abs(U - hi) < tol)


def _oracle_particle(orc, m, seed, k, i, t, x, nn=NN):
    """The particle's S steps with the oracle, and whether a step after the
    first (whose input both sides share exactly) started with a U within
    the threshold tolerance of the states' FP32/FP64 difference."""
    S = m.S
    amb = False
    for s in range(S):
        if s > 0:
            amb |= _near_band(x[:nn])
        x, _ = orc.fhnp_step(m, seed, 2, i, k, (t - 1) * S + s, x)
    return x, amb


@pytest.mark.parametrize("S,fused", [(1, False), (1, True), (4, False), (4, True)])
def test_interval_matches_oracle(pf, orc, torch_mod, S, fused):
    spec = pf_inputs.fhn_paper(J, S=S, eps=0.5)
    M, N, seed, t = 2, 48, 700 + S, 3
    print(f"FH-N network S {S} fused {fused}", flush=True)
    m = orc.Model(spec)
    X0 = _cloud(seed, spec, M, N)
    rng = np.random.default_rng(seed)
    y = (-1.5 + 0.5 * rng.standard_normal(len(spec["obs_idx"]))).astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=fused)
    f.set_particles(0, _dev(X0))
    f.set_interval(t)
    f.run_stages(pf.STAGE_PROPAGATE | pf.STAGE_WEIGHT, _dev(y))
    xb = f.get_predicted(0).cpu().numpy()
    lw = f.get_logweights(0).cpu().numpy()
    f.close()
    n_amb = n_ev = 0
    for k in range(M):
        for i in range(N):
            xo, amb = _oracle_particle(orc, m, seed, k, i, t, X0[k, i].copy())
            if amb:
                n_amb += 1
                continue
            n_ev += int(np.sum(xo[2 * NN:2 * NN + 25] != X0[k, i, 2 * NN:2 * NN + 25]))
            assert np.array_equal(xb[k, i, 2 * NN:], xo[2 * NN:].astype(np.float32)), (k, i)
            assert_rel_close(xb[k, i, :2 * NN], xo[:2 * NN], floor=0.1, what=f"particle {k},{i}")
            assert_rel_close(lw[k, i], orc.loglik(m, xo, y.astype(np.float64)), floor=1.0,
                             what=f"log-weight {k},{i}")
    print(f"exempt {n_amb} of {M * N}; ring slots changed {n_ev}")
    assert n_amb <= 0.05 * M * N
    assert n_ev > 0


# Other grid sizes: each thread owns 4Q consecutive nodes (Q = ceil(J^2 / 1024));
# where J is a multiple of 4Q they lie in one row and the neighbours come from
# row reads (J = 40, Q = 2; J = 64, Q = 4, whose four planes exceed 64 KB of
# LDS), otherwise from per-node reads (J = 30: threads beyond the last node
# idle; J = 36, Q = 2); some particles start with no event in their ring.
@pytest.mark.parametrize("Jg", [30, 36, 40, 64])
def test_interval_other_grids(pf, orc, torch_mod, Jg):
    spec = pf_inputs.fhn_paper(Jg, S=2, eps=0.5)
    nn = Jg * Jg
    M, N, seed, t = 2, 24, 800 + Jg, 3
    print(f"FH-N network J {Jg}", flush=True)
    m = orc.Model(spec)
    X0 = _cloud(seed, spec, M, N, nn)
    X0[:, ::2] = _cloud(seed + 1, spec, M, N, nn, empty_rings=True)[:, ::2]
    rng = np.random.default_rng(seed)
    y = (-1.5 + 0.5 * rng.standard_normal(len(spec["obs_idx"]))).astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=True)
    f.set_particles(0, _dev(X0))
    f.set_interval(t)
    f.step(_dev(y))
    xb = f.get_predicted(0).cpu().numpy()
    lw = f.get_logweights(0).cpu().numpy()
    f.close()
    n_amb = 0
    for k in range(M):
        for i in range(N):
            xo, amb = _oracle_particle(orc, m, seed, k, i, t, X0[k, i].copy(), nn)
            if amb:
                n_amb += 1
                continue
            assert np.array_equal(xb[k, i, 2 * nn:], xo[2 * nn:].astype(np.float32)), (k, i)
            assert_rel_close(xb[k, i, :2 * nn], xo[:2 * nn], floor=0.1, what=f"particle {k},{i}")
            assert_rel_close(lw[k, i], orc.loglik(m, xo, y.astype(np.float64)), floor=1.0,
                             what=f"log-weight {k},{i}")
    assert n_amb <= 0.05 * M * N


# Many particles per workgroup: the launch holds only the resident
# workgroups (a few per CU), so each walks the particles p, p + G, ... with
# the next state prefetched, the planes and rings reused, and the previous
# particle's log-likelihood formed during the next particle's first step.
# 4200 particles (four or five per workgroup); a sample, the last particles
# included, against the oracle.
@pytest.mark.parametrize("S,fused", [(1, True), (2, True), (1, False)])
def test_interval_many_particles_per_workgroup(pf, orc, torch_mod, S, fused):
    spec = pf_inputs.fhn_paper(J, S=S, eps=0.5)
    M, N, seed, t = 2, 2100, 950 + S, 5
    print(f"FH-N network {M}x{N} S {S} fused {fused}", flush=True)
    m = orc.Model(spec)
    X0 = _cloud(seed, spec, M, N)
    X0[:, 1::3] = _cloud(seed + 1, spec, M, N, empty_rings=True)[:, 1::3]
    rng = np.random.default_rng(seed)
    y = (-1.5 + 0.5 * rng.standard_normal(len(spec["obs_idx"]))).astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=fused)
    f.set_particles(0, _dev(X0))
    f.set_interval(t)
    f.run_stages(pf.STAGE_PROPAGATE | pf.STAGE_WEIGHT, _dev(y))
    xb = f.get_predicted(0).cpu().numpy()
    lw = f.get_logweights(0).cpu().numpy()
    f.close()
    picks = sorted(set(rng.integers(0, M * N, 56).tolist()) | {0, 1, M * N - 2, M * N - 1,
                                                                N - 1, N})
    n_amb = n_ev = 0
    for p in picks:
        k, i = divmod(p, N)
        xo, amb = _oracle_particle(orc, m, seed, k, i, t, X0[k, i].copy())
        if amb:
            n_amb += 1
            continue
        n_ev += int(np.sum(xo[2 * NN:2 * NN + 25] != X0[k, i, 2 * NN:2 * NN + 25]))
        assert np.array_equal(xb[k, i, 2 * NN:], xo[2 * NN:].astype(np.float32)), (k, i)
        assert_rel_close(xb[k, i, :2 * NN], xo[:2 * NN], floor=0.1, what=f"particle {k},{i}")
        assert_rel_close(lw[k, i], orc.loglik(m, xo, y.astype(np.float64)), floor=1.0,
                         what=f"log-weight {k},{i}")
    print(f"exempt {n_amb} of {len(picks)}; ring slots changed {n_ev}")
    assert n_amb <= 0.05 * len(picks) + 1
    assert n_ev > 0


def test_prior_draw(pf, orc, torch_mod):
    spec = pf_inputs.fhn_paper(J)
    M, N, seed = 2, 16, 5
    m = orc.Model(spec)
    f = pf.ParticleFilter([spec], [(0, M, N, seed)], fused=True)
    X = f.get_particles(0).cpu().numpy()
    f.close()
    for k in range(M):
        ref = orc.init(m, seed, k, N)
        assert_rel_close(X[k], ref, floor=0.1, what="prior")
        assert np.all(X[k, :, 2 * NN:] == -1.0)


# J = 64 with two steps per observation: the planes take more than 64 KB of
# LDS, and the plane holding U alternates with S even and odd
@pytest.mark.parametrize("Jt,S", [(32, 1), (64, 2)])
def test_truth_simulation_matches_oracle(pf, orc, torch_mod, Jt, S):
    spec = pf_inputs.fhn_paper(Jt, S=S, eps=0.05)
    nn = Jt * Jt
    T, seed = 40, 12
    m = orc.Model(spec)
    xo, yo = orc.simulate(m, seed, T)
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    xt, y = sim.simulate(0, seed, T)
    xt, y = xt.cpu().numpy(), y.cpu().numpy()
    sim.close()
    # compare up to the first step whose start is ambiguous at a threshold
    for t in range(T + 1):
        if t > 0 and _near_band(xo[t - 1, :nn]):
            break
        assert np.array_equal(xt[t, 2 * nn:], xo[t, 2 * nn:].astype(np.float32)), t
        assert_rel_close(xt[t, :2 * nn], xo[t, :2 * nn], floor=0.1, rel=5e-5, what=f"truth {t}")
        if t > 0:
            assert_rel_close(y[t - 1], yo[t - 1], floor=1.0, rel=5e-5, what=f"y {t}")
    assert t >= 10


def _oracle_mse(args):
    seed, T, M, N = args
    import oracle as orc
    spec = pf_inputs.fhn_paper(J)
    m = orc.Model(spec)
    xt, y = orc.simulate(m, 30_000 + seed, T)
    est, _, _, _ = orc.run_ensemble(m, seed, M, N, y.astype(np.float32).astype(np.float64))
    return float(np.mean((est[:, :NN] - xt[1:, :NN]) ** 2))


def test_end_to_end_mse_32_seeds(pf, orc, torch_mod):
    spec = pf_inputs.fhn_paper(J)
    T, M, N = 12, 4, 32
    m = orc.Model(spec)
    gpu = []
    for s in range(1, 33):
        print(f"FH-N network seed {s}", flush=True)
        xt, y = orc.simulate(m, 30_000 + s, T)
        f = pf.ParticleFilter([spec], [(0, M, N, s)], fused=True)
        yd = _dev(y)
        est = np.zeros((T, spec["dx"]))
        for t in range(T):
            f.step(yd[t])
            est[t] = f.estimate()[0].cpu().numpy()
        f.close()
        gpu.append(float(np.mean((est[:, :NN] - xt[1:, :NN]) ** 2)))
    with cf.ThreadPoolExecutor(8) as pool:
        ora = list(pool.map(_oracle_mse, [(s, T, M, N) for s in range(1, 33)]))
    gpu, ora = np.array(gpu), np.array(ora)
    se = ora.std(ddof=1) / np.sqrt(32)
    print(f"MSE(U) gpu {gpu.mean():.5f} oracle {ora.mean():.5f} (2 SE = {2 * se:.5f})")
    assert abs(gpu.mean() - ora.mean()) <= 2 * se


def test_batch_members_equal_runs_alone(pf, torch_mod):
    specs = [pf_inputs.fhn_paper(J), pf_inputs.lorenz63()]
    ens = [(0, 2, 40, 31), (1, 3, 300, 32), (0, 1, 64, 33, 0, "systematic", 0.5)]
    T = 3
    sim = pf.ParticleFilter(specs, [(0, 1, 1, 1), (1, 1, 1, 1)], fused=True)
    ys = [sim.simulate(e[0], 60 + i, T)[1] for i, e in enumerate(ens)]
    sim.close()
    y_all = torch_mod.cat(ys, dim=1).contiguous()
    for graph in (False, True):
        print(f"FH-N network batch graph={graph}", flush=True)
        f = pf.ParticleFilter(specs, ens, fused=True, graph=graph)
        if graph:
            f.set_observations(y_all)
        for t in range(T):
            f.step(None if graph else y_all[t])
        batch = [f.get_predicted(e).cpu().numpy() for e in range(len(ens))]
        mean = f.estimate()[0].cpu().numpy()
        f.close()
        off = 0
        for e, d in enumerate(ens):
            g = pf.ParticleFilter([specs[d[0]]], [(0,) + tuple(d[1:])], fused=True)
            for t in range(T):
                g.step(ys[e][t].contiguous())
            assert np.array_equal(batch[e], g.get_predicted(0).cpu().numpy()), e
            dx = specs[d[0]]["dx"]
            assert np.array_equal(mean[off:off + dx], g.estimate()[0].cpu().numpy()), e
            off += dx
            g.close()


@pytest.mark.parametrize("N", [64, 2100])
def test_auxiliary_filter_interval_matches_oracle(pf, orc, torch_mod, N):
    # the paper's filter on its network: pilot = the noise-free continuation
    # with the active stimuli of the ring (eps = 0: no new events, so no
    # threshold decision is involved), first stage, propagation, carried
    # second-stage weights (N = 2100: several particles per workgroup in
    # both the pilot and the propagation kernel)
    from pf_testlib import rel_close
    spec = pf_inputs.fhn_paper(J, S=2, eps=0.0)
    M, seed, t = 2, 909, 4
    print(f"FH-N network auxiliary {M}x{N}", flush=True)
    m = orc.Model(spec)
    X0 = _cloud(seed, spec, M, N)
    rng = np.random.default_rng(seed)
    lwc0 = rng.standard_normal((M, N)) * 0.5
    lwc0 = np.log(N * np.exp(lwc0) / np.exp(lwc0).sum(axis=1, keepdims=True)).astype(np.float32)
    y = (-1.5 + 0.5 * rng.standard_normal(len(spec["obs_idx"]))).astype(np.float32)
    f = pf.ParticleFilter([spec], [(0, M, N, seed, pf.ENS_AUXILIARY)], fused=True)
    f.set_particles(0, _dev(X0))
    f.set_carried_logweights(0, _dev(lwc0))
    f.set_interval(t)
    f.step(_dev(y))
    xb = f.get_predicted(0).cpu().numpy()
    lw = f.get_logweights(0).cpu().numpy()
    lwc = f.get_carried_logweights(0).cpu().numpy()
    f.close()
    for k in range(M):
        r = orc.apf_interval(m, seed, k, t, X0[k], lwc0[k].astype(np.float64),
                             y.astype(np.float64), 0.0, "multinomial")
        okx = rel_close(xb[k], r["X"], floor=0.1).all(axis=1)
        okl = rel_close(lw[k], r["lw"], floor=1.0)
        ok = okx & okl
        assert ok.mean() >= 0.98, (k, ok.mean())
        assert rel_close(lwc[k][ok], r["lwc"][ok], floor=1.0).all(), k
