"""Workload definitions and seeded synthetic inputs.

This module is shared by the tests, the benchmark and the oracle wrappers, and
holds none of the filter's arithmetic: it only states the model constants,
shapes and seeds of each workload, and draws seeded test inputs (particle
clouds, log-weights) with numpy's generator.  Random numbers that the method
itself consumes (Euler noise, prior draws, resampling uniforms) are never
drawn here; both implementations generate them from Philox4x32-10 counters.

Model dictionaries use the keys:
  kind       'ou1d' | 'lorenz63' | 'fhn'
  dx, J, S   state dimension, grid side (FH-N), Euler steps per observation
  h          Euler step
  params     OU: (theta,) | L63: (s, r, b) | FH-N: (a, D, eps, gamma)
  noise_sd   diffusion coefficient per variable class (x sqrt(h) per step)
  obs_idx    observed state indices; obs_var observation noise variance
  prior_mean, prior_sd   tau_0 = N(prior_mean, diag(prior_sd^2))
"""
from __future__ import annotations

import numpy as np


def lorenz63(obs_every: int = 40) -> dict:
    """Stochastic Lorenz 63 (Sec. 4.1 model, constants of the 4x256 workload):
    s=10, r=28, b=8/3, h=1e-3, diffusion 0.5 per component, x1 and x3
    observed every 40 steps with variance 0.5, prior N((-5.9,-5.5,24.5), I)."""
    return dict(kind="lorenz63", dx=3, J=0, S=obs_every, h=1e-3,
                params=(10.0, 28.0, 8.0 / 3.0), noise_sd=(0.5, 0.5),
                obs_idx=[0, 2], obs_var=0.5,
                prior_mean=[-5.9, -5.5, 24.5], prior_sd=[1.0, 1.0, 1.0])


def lorenz63_paper() -> dict:
    """The stochastic Lorenz 63 system of the paper's own experiment (Sec. 4.1,
    eqs. eqDiscreteLorenz-1..3 and eqObservLorenz): s=10, r=28, b=8/3, Euler
    step T_d = 1e-3 with unit diffusion (sqrt(T_d) U per component), x1
    observed every 100 steps with noise variance 1/2, prior N(x*, 10 I) with
    x* = (-10.2410, -1.3984, 23.6752) -- the third component read with a
    positive sign: the printed -23.6752 is off the attractor, where x3 > 0
    on every trajectory of the deterministic system the mean was taken from."""
    return dict(kind="lorenz63", dx=3, J=0, S=100, h=1e-3,
                params=(10.0, 28.0, 8.0 / 3.0), noise_sd=(1.0, 1.0),
                obs_idx=[0], obs_var=0.5,
                prior_mean=[-10.2410, -1.3984, 23.6752], prior_sd=[10.0 ** 0.5] * 3)


# the paper's Lorenz experiment (Sec. 4.2, 4.3): M = 20 filters, N per filter,
# the centralised filter with K = M N, 200 observations, 100 runs per N, the
# posterior-mean proxy from one filter of J = 1e5 particles
PAPER_L63 = dict(M=20, Ns=(100, 200, 400, 600, 800, 1000), T=200, runs=100, proxy_J=100000)


def fhn_obs_nodes(J: int) -> list:
    """Every 4th node in each direction, rows/cols 2, 6, 10, ... (0-based),
    row-major; returned as v-plane state indices i*J + j."""
    rows = list(range(2, J, 4))
    return [i * J + j for i in rows for j in rows]


def fhn(J: int = 40, S: int = 20) -> dict:
    """Classical stochastic FitzHugh-Nagumo grid: dv = (v(v-0.1)(1-v) - w +
    0.5 lap v)dt + 0.05 dW, dw = 0.01 (v - 0.5 w) dt + 0.05 dW, h = 0.05,
    no-flux 5-point Laplacian, v observed at every 4th node with variance 0.01.
    Prior: v = 1 on the 5x5 corner block (a stimulus that launches a wave),
    v = 0 elsewhere, w = 0, all with sd 0.05."""
    nn = J * J
    mean = np.zeros(2 * nn)
    for i in range(min(5, J)):
        for j in range(min(5, J)):
            mean[i * J + j] = 1.0
    return dict(kind="fhn", dx=2 * nn, J=J, S=S, h=0.05,
                params=(0.1, 0.5, 0.01, 0.5), noise_sd=(0.05, 0.05),
                obs_idx=fhn_obs_nodes(J), obs_var=0.01,
                prior_mean=mean.tolist(), prior_sd=[0.05] * (2 * nn))


def fhn_paper_obs_nodes(J: int = 32) -> list:
    """The paper's observation zones (Sec. 5.2): a 5 x 5 grid of 2 x 2 node
    squares, equally spaced -- read as top-left corners at rows and columns
    6k + 3 (k = 0..4, 0-based), which leaves three unobserved rows and
    columns on each border of the 32 x 32 grid; row-major U-plane indices."""
    starts = [6 * k + 3 for k in range(5)]
    rows = sorted(r + d for r in starts for d in (0, 1))
    return [i * J + j for i in rows for j in rows]


def fhn_paper(J: int = 32, S: int = 1, eps: float = 1e-3) -> dict:
    """The paper's modified stochastic FitzHugh-Nagumo network (Sec. 5.1, 5.2):
    p3(u) = 3.6 u - u^3 (read with a negative leading coefficient), coupling
    (1/D) sum of the 4 neighbours' U with 1/D = 4.5e-3, recovery (2.1, -0.6,
    0.6), noise variance 1/2 on U only, T_d = 5e-3; random stimuli of
    amplitude 200 for l0 = 25 steps at a uniform node of the region where
    U (or a neighbour's U) lies in (-1.8, -1.6), with probability eps = 1e-3
    per step; periodic forcing of amplitude 200 every 20 time units (4000
    steps) on the 2 x 2 corner block, read as a pulse of l0 steps; U observed
    at every step on the 100 nodes of the 2 x 2 zones with variance 1/2.
    Prior: U, V near the node's rest point (-1.033, -2.616) with sd 0.05, no
    past stimuli.  The state is U, V and the ring of the last l0 stimulus
    events (padded to 28 entries)."""
    nn = J * J
    l0 = 25
    ring = 4 * ((l0 + 3) // 4)
    mean = [-1.0332] * nn + [-2.6162] * nn + [-1.0] * ring
    sd = [0.05] * (2 * nn) + [0.0] * ring
    return dict(kind="fhn_paper", dx=2 * nn + ring, J=J, S=S, h=5e-3,
                params=(3.6, 4.5e-3, 2.1, -0.6), noise_sd=(0.5 ** 0.5, 0.0),
                params_ext=(0.6, 200.0, eps, -1.8, -1.6, float(l0), 4000.0, float(l0)),
                obs_idx=fhn_paper_obs_nodes(J), obs_var=0.5,
                prior_mean=mean, prior_sd=sd)


# the paper's FH-N network experiment (Sec. 5.3): M = 10 filters with N per
# filter (the paper's auxiliary filters, here bootstrap filters)
PAPER_FHN = dict(M=10, Ns=(100, 500, 1000, 2000, 5000))


def ou1d(theta=1.0, sd=1.0, h=0.01, S=10, obs_var=0.05, prior_mean=0.0,
         prior_sd=1.0) -> dict:
    """1-D Ornstein-Uhlenbeck test model, x' = x - theta h x + sd sqrt(h) z,
    observed directly every S steps (linear-Gaussian: exact Kalman filter)."""
    return dict(kind="ou1d", dx=1, J=0, S=S, h=h, params=(theta,),
                noise_sd=(sd, sd), obs_idx=[0], obs_var=obs_var,
                prior_mean=[prior_mean], prior_sd=[prior_sd])


# ------------------------------------------------------------- workloads -----
WORKLOADS = {
    # name: (model factory, M, N, T)
    "l63_4x256": (lorenz63, 4, 256, 100),
    # the paper's own Lorenz experiment (largest ensemble, M = 20 x N = 1000)
    "l63_paper": (lorenz63_paper, 20, 1000, 200),
    "l63_sweep_M1": (lorenz63, 1, 1 << 20, 1000),
    "l63_sweep_M16": (lorenz63, 16, 1 << 16, 1000),
    "l63_sweep_M256": (lorenz63, 256, 1 << 12, 1000),
    "l63_sweep_M4096": (lorenz63, 4096, 1 << 8, 1000),
    "fhn40_64x512": (fhn, 64, 512, 200),
    "fhn20_4x64": (lambda: fhn(20), 4, 64, 20),
    # learned proposal, compared with the bootstrap filter at N = 512
    "fhn40_learned_64x128": (fhn, 64, 128, 200),
    # the paper's FH-N network, its largest ensemble (M = 10 x N = 5000)
    "fhn_paper_10x5000": (fhn_paper, 10, 5000, 300),
    # uneven serving mix (see mixed_batch): 1024 Lorenz + 32 FH-N 20 x 20 tenants
    "mix_l63x1024_fhn20x32": (None, None, None, 100),
}

# training of the learned proposal for the fhn40 learned workload: 1e4
# one-interval trajectories (100 model runs x 100 intervals), Adam steps of
# 4096 tiles of 16 nodes with the learning rate stepped down
LEARNED_TRAINING = dict(n_runs=100, run_len=100, batch_tiles=4096,
                        schedule=((2000, 3e-4), (2000, 1e-4), (2000, 3e-5)), seed=21)


def mixed_batch(seed: int = 1, n_l63: int = 1024, n_fhn: int = 32):
    """Uneven serving-style batch: n_l63 Lorenz filters with N log-uniform in
    [64, 8192] and n_fhn FH-N 20x20 filters with N in {128, 256, 512}; each
    filter is its own ensemble (M = 1) with its own seed."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_l63)
    n_l = np.floor(np.exp(np.log(64.0) + u * np.log(128.0))).astype(int)
    n_l = np.clip(n_l, 64, 8192)
    n_f = rng.choice([128, 256, 512], size=n_fhn)
    return [int(v) for v in n_l], [int(v) for v in n_f]


# ------------------------------------------------------------- test inputs ---
def particles(seed: int, model: dict, M: int, N: int, spread: float = 1.0) -> np.ndarray:
    """Seeded particle cloud [M, N, dx] (float64) around the prior mean."""
    rng = np.random.default_rng(seed)
    mean = np.asarray(model["prior_mean"], dtype=np.float64)
    sd = np.asarray(model["prior_sd"], dtype=np.float64)
    return mean + spread * sd * rng.standard_normal((M, N, mean.size))


def logweights(seed: int, M: int, N: int, scale: float = 5.0) -> np.ndarray:
    """Seeded log-weights [M, N] (float32 values) with a spread of `scale`."""
    rng = np.random.default_rng(seed)
    return (-scale * rng.random((M, N)) ** 2 * 4.0).astype(np.float32)
