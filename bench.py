"""Benchmark: particle-steps/s of the independent-ensemble bootstrap filter on
one MI355X.

A step is one observation interval of the whole hot path (S Euler-Maruyama
steps of every particle, weighting, normalisation, multinomial resampling,
gather and the ensemble estimate) over one batch; the default workload is the
Lorenz 63 time-error sweep split M = 256 filters x N = 4096 particles
(K = 2^20 particles, S = 40 Euler steps per interval).  Observations are
synthetic: the library's own truth simulator on the GPU.

Prints one JSON line with the throughput, the dominant kernel's roofline
(timed live with HIP events around its launches in every PROF_EVERY-th timed
interval) and the FP64 oracle
timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import pf_inputs  # noqa: E402

# ---------------------------------------------------------------------------
# Roofline constants of one MI355X (256 CUs, 2.4 GHz).
#   HBM3E peak 8 TB/s.
#   VALU: a full-rate 32-bit instruction (FP32 FMA/add/mul, bit ops) issues
#   for 128 lanes per CU per clock, i.e. 7.86e13 lane-ops/s, which is the
#   published 157.3 TFLOP/s FP32 at 2 FLOP per FMA.  Work is counted in
#   full-rate issue slots and reported in FMA-equivalent FLOP (2 per slot);
#   half-rate instructions (32x32-bit integer multiply, v_mad_u64_u32, FP64
#   FMA, int->float conversion) take 2 slots, transcendentals (log2, sqrt,
#   sin, cos, exp) take 4 -- the rates measured on the device.
HBM_PEAK_GBS = 8000.0
VALU_SLOTS_PER_S = 256 * 128 * 2.4e9
FLOP_PER_SLOT = 2.0

# Algorithmic VALU slots of one Philox4x32-10 call (10 rounds x (2 wide
# products x 2 + 2 three-way XORs x 1: gfx950's v_bitop3_b32 takes a ^ b ^ c
# in one instruction, which the register-only probe places at ~1.4 slots, so
# 1 is the lower count) and of one Box-Muller pair (2 uniforms x 3 -- the
# 23 random bits moved into a float's mantissa, one subtraction --, log2,
# sqrt, sin, cos x 4, 3 multiplies).
PHILOX_SLOTS = 60.0
BOXMULLER_SLOTS = 25.0
# The dominant kernel's launches are bracketed by HIP events on every
# PROF_EVERY-th interval of the timed region only: an event pair costs the
# stream ~6 us (the Lorenz 256 x 4096 interval measured 0.104 ms without and
# 0.110 ms with a pair around every propagation launch), which would slow
# the very intervals whose throughput is reported.
PROF_EVERY = 8

# intervals of the untimed accuracy pass
ACCURACY_INTERVALS = 220

# Lorenz 63 particle-step: 3 Philox calls per 4 steps, 1.5 Box-Muller pairs,
# drift (7) and the Euler update (2 FMAs per component).
L63_SLOTS_PER_PARTICLE_STEP = 0.75 * PHILOX_SLOTS + 1.5 * BOXMULLER_SLOTS + 7 + 6
# FH-N node-step: one Philox call per 2 nodes, one Box-Muller pair, the
# 4-neighbour Laplacian (7), reaction and recovery drifts (8), 2 x 2 FMAs.
FHN_SLOTS_PER_NODE_STEP = 0.5 * PHILOX_SLOTS + BOXMULLER_SLOTS + 7 + 8 + 4
# FH-N streaming Euler step: every node's v and w read and written once.
FHN_BYTES_PER_NODE_STEP = 16.0

# Learned proposal: the MLP 22 -> 64 -> 64 -> 2 per node and Euler step,
# 2 (22*64 + 64*64 + 64*2) FLOP, against the dense bfloat16 MFMA peak.
MLP_FLOP_PER_NODE_STEP = 2.0 * (22 * 64 + 64 * 64 + 64 * 2)
BF16_MFMA_PEAK_TFLOPS = 2500.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB; fetch scaled x2, write x1 by the same counters on a 1 GiB
# copy), recorded in profiles/hbm_counters_fhn_stream_step_and_lorenz_propagation.md
# for the kernels as they are now.
MEASURED_TRAFFIC_BYTES = {
    ("lorenz63", "fused", 256, 4096): (15618 + 16384) * 1024,
    ("fhn", "plain", 64, 512): (409688 + 409610) * 1024,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed intervals first (default: 500 for the Lorenz workloads, whose "
                         "first few hundred intervals -- 20-40 ms of load -- measured ~6%% slower "
                         "than later ones; 200 for the mix; 20 for the FH-N workloads, whose "
                         "intervals are long and whose tracked wave is a transient)")
    ap.add_argument("--workload", default="l63_sweep_M256", choices=sorted(pf_inputs.WORKLOADS))
    ap.add_argument("--path", default="fused", choices=["plain", "fused", "graph"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0 disables it)")
    ap.add_argument("--accuracy", type=int, default=1,
                    help="1: after the timed run, an untimed pass that reports the MSE of the "
                         "ensemble estimate against the simulated truth (and, for the Lorenz "
                         "sweep, against a 64 x 2^20-particle reference filter)")
    a = ap.parse_args()
    if a.warmup is None:
        kind = pf_inputs.WORKLOADS[a.workload][0]
        a.warmup = (200 if a.workload.startswith("mix") else
                    500 if kind is pf_inputs.lorenz63 else 20)
    return a


def _oracle_worker(args):
    spec, seed, filt, N, intervals, y = args
    import oracle
    m = oracle.Model(spec)
    X = oracle.init(m, seed, filt, N)
    lz = 0.0
    t0 = time.perf_counter()
    for t in range(1, intervals + 1):
        r = oracle.filter_interval(m, seed, filt, t, X, y[t - 1], lz)
        X, lz = r["X"], r["logZ"]
    return time.perf_counter() - t0


def cpu_baseline(spec, M, N, y_host, target_s):
    """The FP64 oracle on a bounded sample of the workload: whole filters of
    the same N for a few intervals, spread over the host cores the way the
    paper spreads filters over cores (each filter single-threaded)."""
    import concurrent.futures as cf
    import oracle
    oracle.lib()
    cores = max(1, min(16, os.cpu_count() or 1))
    # calibrate with one interval of one filter
    dt1 = _oracle_worker((spec, 1, 0, N, 1, y_host))
    per_filter_interval = max(dt1, 1e-6)
    intervals = max(1, min(len(y_host), int(target_s / per_filter_interval / max(1, min(M, cores)))))
    n_filters = min(M, cores)
    jobs = [(spec, 1, f, N, intervals, y_host) for f in range(n_filters)]
    t0 = time.perf_counter()
    # one thread per filter: the oracle's C calls release the GIL
    with cf.ThreadPoolExecutor(n_filters) as pool:
        list(pool.map(_oracle_worker, jobs))
    wall = time.perf_counter() - t0
    steps = n_filters * intervals * N * spec["S"]
    return {"value": steps / wall, "unit": "particle-steps/s", "cores": n_filters,
            "wall_s": wall,
            "kind": "oracle",
            "sample": f"{n_filters} filters x N={N} x {intervals} intervals "
                      f"({steps:.3g} particle-steps, FP64, one filter per core)"}


def _run_filter(pf, torch, spec, M, N, flags, params, y, warmup, steps, est_out):
    """Warm-up, then `steps` timed intervals with the ensemble estimate of
    each kept on the device; returns (ms, kernel ms, kernel launches)."""
    import ctypes as C
    f = pf.ParticleFilter([spec], [(0, M, N, 1, flags)], fused=True)
    if params is not None:
        f.set_proposal(0, params)
    stream = torch.cuda.current_stream()
    for t in range(warmup):
        f.step(y[t])
    torch.cuda.synchronize()
    f.read_profile()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dx = spec["dx"]
    lz = torch.empty(M, dtype=torch.float64, device="cuda")
    e0.record(stream)
    for k, t in enumerate(range(warmup, warmup + steps)):
        f.set_profiling(k % PROF_EVERY == 0)
        f.step(y[t])
        pf._check(pf.lib().pf_estimate(f._ctx, C.c_void_p(est_out[k].data_ptr()), None,
                                       C.c_void_p(lz.data_ptr()), None, pf._stream(None)))
    e1.record(stream)
    torch.cuda.synchronize()
    f.set_profiling(False)
    k_ms, k_n = f.read_profile()
    del dx
    return e0.elapsed_time(e1), k_ms, k_n


def _estimates(pf, torch, spec, M, N, y, T):
    """Untimed: a fresh fused filter over y[0:T]; the ensemble estimate of
    every interval, [T][dx] on the device."""
    import ctypes as C
    f = pf.ParticleFilter([spec], [(0, M, N, 1)], fused=True)
    est = torch.empty((T, spec["dx"]), dtype=torch.float64, device="cuda")
    lz = torch.empty(M, dtype=torch.float64, device="cuda")
    for t in range(T):
        f.step(y[t])
        pf._check(pf.lib().pf_estimate(f._ctx, C.c_void_p(est[t].data_ptr()), None,
                                       C.c_void_p(lz.data_ptr()), None, pf._stream(None)))
    torch.cuda.synchronize()
    del f
    return est


def accuracy(pf, torch, spec, M, N, xt, y, T, reference):
    """MSE of the ensemble estimate of x_t against the simulated truth over
    T intervals (FH-N: the v nodes), the paper's C_ipf = 1/M + 1/N, and for
    the Lorenz sweep the MSE against the estimate of 64 filters x 2^20
    particles on the same observations (variance ~ 1/(64 * 2^20), bias
    ~ 2^-40), which isolates the ensemble's own error (Thm 1, Cor. 2)."""
    comps = spec["J"] ** 2 if spec["kind"] == "fhn" else spec["dx"]
    est = _estimates(pf, torch, spec, M, N, y, T)
    truth = xt[1:T + 1, :comps].double()
    out = {"intervals": T, "components": "v nodes" if spec["kind"] == "fhn" else "x1, x2, x3",
           "mse_vs_truth": torch.mean((est[:, :comps] - truth) ** 2).item(),
           "c_ipf": 1.0 / M + 1.0 / N}
    if reference:
        ref = _estimates(pf, torch, spec, 64, 1 << 20, y, T)
        out["mse_vs_reference_64x2^20"] = torch.mean((est[:, :comps] - ref[:, :comps]) ** 2).item()
        out["reference_mse_vs_truth"] = torch.mean((ref[:, :comps] - truth) ** 2).item()
        del ref
    del est
    torch.cuda.empty_cache()
    return out


def cpu_baseline_learned(spec, params, y_host, target_s):
    """The FP64 oracle of the learned filter (its bfloat16-rounding mode, the
    GPU's arithmetic) on a bounded sample: one filter per host core, each a
    few particles through the first interval."""
    import concurrent.futures as cf
    import oracle
    oracle.lib()
    m = oracle.Model(spec)
    cores = max(1, min(16, os.cpu_count() or 1))

    def work(job):
        filt, n = job
        X = oracle.init(m, 1, filt, n)
        t0 = time.perf_counter()
        oracle.filter_interval_learned(m, params, 1, filt, 1, X, y_host[0], 0.0)
        return time.perf_counter() - t0

    dt1 = max(work((0, 1)), 1e-6)
    n_per = max(1, int(target_s / dt1))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as pool:
        list(pool.map(work, [(f, n_per) for f in range(cores)]))
    wall = time.perf_counter() - t0
    steps = cores * n_per * spec["S"]
    return {"value": steps / wall, "unit": "particle-steps/s", "cores": cores, "wall_s": wall,
            "kind": "oracle",
            "sample": f"{cores} filters x N={n_per} x 1 interval of the learned filter "
                      f"({steps} particle-steps of {spec['J']}x{spec['J']} nodes, FP64)"}


def learned_main(a):
    """FH-N 40 x 40 with the learned proposal (M = 64 x N = 128) against the
    bootstrap filter at N = 512 on the same GPU-simulated observations: wall
    time per assimilated observation and MSE of v against the truth; the
    training is timed on its own."""
    import torch
    import paper_1407_8071_amd as pf
    factory, M, N, _ = pf_inputs.WORKLOADS[a.workload]
    spec = factory()
    tc = pf_inputs.LEARNED_TRAINING
    torch.cuda.set_device(0)
    # training on model-simulated trajectories
    t0 = time.perf_counter()
    tr = pf.Trainer(spec, tc["n_runs"], tc["run_len"], tc["batch_tiles"], seed=tc["seed"])
    tr.data()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    rng = np.random.default_rng(1)
    n_in = 22
    params = np.zeros(pf.mlp_nparams(n_in, 2), np.float32)
    params[:64 * n_in] = rng.standard_normal(64 * n_in) * np.sqrt(2 / n_in)
    o = 64 * n_in + 64
    params[o:o + 4096] = rng.standard_normal(4096) * np.sqrt(2 / 64)
    p = torch.from_numpy(params).cuda()
    t1 = time.perf_counter()
    n_steps = 0
    for n, lr in tc["schedule"]:
        tr.desc.lr = lr
        tr.steps(p, n)
        n_steps += n
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del tr
    torch.cuda.empty_cache()
    # observations from the library's truth simulator
    T = a.warmup + a.steps
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    xt, y = sim.simulate(0, 1, T)
    torch.cuda.synchronize()
    nn = spec["J"] ** 2
    truth = xt[1 + a.warmup:1 + T, :nn].double()
    res = {}
    runs = (("learned", N, pf.ENS_LEARNED, p), ("bootstrap_N%d" % N, N, 0, None),
            ("bootstrap_N%d" % (4 * N), 4 * N, 0, None),
            ("bootstrap_N%d" % (16 * N), 16 * N, 0, None))
    for name, n_p, flags, prm in runs:
        est = torch.empty((a.steps, spec["dx"]), dtype=torch.float64, device="cuda")
        ms, k_ms, k_n = _run_filter(pf, torch, spec, M, n_p, flags, prm, y, a.warmup, a.steps, est)
        mse = torch.mean((est[:, :nn] - truth) ** 2).item()
        psteps = M * n_p * spec["S"] * a.steps
        res[name] = {"M": M, "N": n_p, "ms_per_interval": ms / a.steps, "mse_v": mse,
                     "particle_steps_per_s": psteps / (ms / 1e3),
                     "kernel_avg_us": k_ms / max(k_n, 1) * 1e3, "kernel_launches": k_n}
        torch.cuda.empty_cache()
    L = res["learned"]
    cpu = None
    if a.cpu_seconds > 0:
        cpu = cpu_baseline_learned(spec, p.double().cpu().numpy(), y.double().cpu().numpy(),
                                   a.cpu_seconds)
    k_avg_s = L["kernel_avg_us"] / 1e6
    flop = MLP_FLOP_PER_NODE_STEP * nn * spec["S"] * M * N
    achieved = flop / k_avg_s / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                "kernel": "k_grid_steps_learned", "algorithmic_flop_per_launch": flop,
                "kernel_avg_us": L["kernel_avg_us"], "launches": L["kernel_launches"],
                "timed_intervals": f"every {PROF_EVERY}th of the timed region"}
    line = {
        "metric": "particle-steps/s", "value": L["particle_steps_per_s"],
        "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": L["ms_per_interval"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 MFMA network, f32 filter",
        "data": "synthetic (GPU-simulated truth and observations; model-simulated training paths)",
        "config": {"workload": a.workload, "model": "fhn", "J": spec["J"], "M": M, "N": N,
                   "S": spec["S"], "path": "fused"},
        "learned": L, "bootstrap": [v for k, v in res.items() if k != "learned"],
        "learned_speedup_vs_bootstrap_N%d" % (4 * N):
            res["bootstrap_N%d" % (4 * N)]["ms_per_interval"] / L["ms_per_interval"],
        "training": {"trajectories": tc["n_runs"] * tc["run_len"], "adam_steps": n_steps,
                     "rows_per_step": 16 * tc["batch_tiles"], "data_s": t_data, "train_s": t_train},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def _mix_oracle_worker(args):
    spec, seed, N, intervals, y = args
    import oracle
    m = oracle.Model(spec)
    X = oracle.init(m, seed, 0, N)
    lz = 0.0
    t0 = time.perf_counter()
    for t in range(1, intervals + 1):
        r = oracle.filter_interval(m, seed, 0, t, X, y[t - 1], lz)
        X, lz = r["X"], r["logZ"]
    return time.perf_counter() - t0, N * spec["S"] * intervals


def mix_main(a):
    """The uneven serving mix: 1024 Lorenz 63 tenants with N log-uniform in
    [64, 8192] and 32 FH-N 20 x 20 tenants with N in {128, 256, 512}, each an
    ensemble of one filter with its own seed and observations, advanced by
    one graph-replayed fused interval per observation under the autotuner's
    launch plan.  Also times the plain multi-launch path on a few intervals."""
    import concurrent.futures as cf
    import torch
    import paper_1407_8071_amd as pf
    n_l, n_f = pf_inputs.mixed_batch(1)
    specs = [pf_inputs.lorenz63(), pf_inputs.fhn(20)]
    ens = [(0, 1, n, 1000 + i) for i, n in enumerate(n_l)] + \
          [(1, 1, n, 5000 + i) for i, n in enumerate(n_f)]
    torch.cuda.set_device(0)
    T = a.warmup + a.steps
    # truth and observations of every tenant on the GPU (the library's simulator)
    sim = pf.ParticleFilter(specs, [(0, 1, 1, 1), (1, 1, 1, 1)], fused=True)
    ys = []
    for i, (mi, _, _, seed) in enumerate(ens):
        _, y = sim.simulate(mi, seed, T)
        ys.append(y)
    y_all = torch.cat(ys, dim=1).contiguous()
    del sim
    psteps_interval = sum(n * specs[mi]["S"] for (mi, _, n, _) in ens)
    l63_ps = sum(n * 40 for n in n_l)
    fhn_ps = sum(n * 20 for n in n_f)
    # autotuned launch plan, then graph replay of the staged observations
    f = pf.ParticleFilter(specs, ens, graph=True)
    t0 = time.perf_counter()
    tuning = f.autotune(y_all[0], reps=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    f.set_observations(y_all)
    for t in range(a.warmup):
        f.step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t1 = time.perf_counter()
    e0.record(stream)
    for t in range(a.steps):
        f.step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms = e0.elapsed_time(e1)
    est = f.estimate()[0].cpu().numpy()
    assert np.all(np.isfinite(est)), "non-finite estimate"
    del f
    # the propagation kernels (Lorenz tiles + batched FH-N steps) with events,
    # on a directly launched fused context with the same plan
    g = pf.ParticleFilter(specs, ens, fused=True)
    g.set_tuning(tuning)
    for t in range(3):
        g.step(y_all[t])
    torch.cuda.synchronize()
    g.read_profile()
    g.set_profiling(True)
    nprof = min(20, T - 3)
    for t in range(3, 3 + nprof):
        g.step(y_all[t])
    torch.cuda.synchronize()
    g.set_profiling(False)
    k_ms, k_n = g.read_profile()
    del g
    slots = (L63_SLOTS_PER_PARTICLE_STEP * l63_ps + FHN_SLOTS_PER_NODE_STEP * 400 * fhn_ps) * nprof
    achieved = slots * FLOP_PER_SLOT / (k_ms / 1e3) / 1e12
    peak = VALU_SLOTS_PER_S * FLOP_PER_SLOT / 1e12
    lorenz_kernel = ("k_filter_wg (whole Lorenz intervals, resampling included)"
                     if tuning["vec_single_kernel"] else "k_vec_prop_batched")
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel": lorenz_kernel + " + k_grid_steps (batched FH-N), summed; "
                          "algorithmic work = propagation slots only",
                "algorithmic_slots_per_interval": slots / nprof,
                "kernel_ms_per_interval": k_ms / nprof, "launches": k_n}
    # the plain path: one kernel per method step and ensemble
    pl = pf.ParticleFilter(specs, ens, fused=False)
    pl.step(y_all[0])
    torch.cuda.synchronize()
    n_plain = 3
    q0 = torch.cuda.Event(enable_timing=True)
    q1 = torch.cuda.Event(enable_timing=True)
    q0.record(stream)
    for t in range(1, 1 + n_plain):
        pl.step(y_all[t])
    q1.record(stream)
    torch.cuda.synchronize()
    plain_ms = q0.elapsed_time(q1) / n_plain
    del pl
    cpu = None
    if a.cpu_seconds > 0:
        import oracle
        oracle.lib()
        yh = [y.double().cpu().numpy() for y in ys]
        cores = max(1, min(16, os.cpu_count() or 1))
        # a bounded sample: the first tenants of each model, a few intervals
        sample = list(range(12)) + list(range(len(n_l), len(n_l) + 4))
        jobs = [(specs[ens[i][0]], ens[i][3], ens[i][2], 2, yh[i]) for i in sample]
        tc = time.perf_counter()
        with cf.ThreadPoolExecutor(cores) as pool:
            res = list(pool.map(_mix_oracle_worker, jobs))
        cw = time.perf_counter() - tc
        steps = sum(r[1] for r in res)
        cpu = {"value": steps / cw, "unit": "particle-steps/s", "cores": min(cores, len(jobs)),
               "wall_s": cw, "kind": "oracle",
               "sample": f"12 Lorenz + 4 FH-N tenants of the mix x 2 intervals "
                         f"({steps:.3g} particle-steps, FP64, one filter per core)"}
    line = {
        "metric": "particle-steps/s", "value": psteps_interval * a.steps / (ms / 1e3),
        "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated truth and observations per tenant)",
        "config": {"workload": a.workload, "tenants_l63": len(n_l), "tenants_fhn20": len(n_f),
                   "particles_l63": int(sum(n_l)), "particles_fhn": int(sum(n_f)),
                   "particle_steps_per_interval": psteps_interval, "path": "graph",
                   "tuning": tuning, "tune_s": tune_s, "wall_s": wall},
        "plain_path_ms_per_interval": plain_ms,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the ensemble would shard by whole filters, one group of filters per GPU)", file=sys.stderr)
        sys.exit(2)
    if a.workload == "fhn40_learned_64x128":
        learned_main(a)
        return
    if a.workload == "mix_l63x1024_fhn20x32":
        mix_main(a)
        return
    import torch
    import paper_1407_8071_amd as pf

    factory, M, N, T_cfg = pf_inputs.WORKLOADS[a.workload]
    spec = factory()
    grid = spec["kind"] == "fhn"
    torch.cuda.set_device(0)
    f = pf.ParticleFilter([spec], [(0, M, N, 1)], fused=(a.path == "fused"),
                          graph=(a.path == "graph"))
    T = a.warmup + a.steps
    xt, y = f.simulate(0, 1, T)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    graph = a.path == "graph"
    if graph:
        f.set_observations(y)
    for t in range(a.warmup):
        f.step(None if graph else y[t])
    torch.cuda.synchronize()
    f.read_profile()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for k, t in enumerate(range(a.warmup, T)):
        f.set_profiling(k % PROF_EVERY == 0)
        f.step(None if graph else y[t])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    f.set_profiling(False)
    k_ms, k_n = f.read_profile()
    f.sync()
    est = f.estimate()[0].cpu().numpy()
    assert np.all(np.isfinite(est)), "non-finite estimate"

    S = spec["S"]
    nodes = spec["J"] ** 2 if grid else 1
    psteps = M * N * S * a.steps
    ms_per_step = ms / a.steps
    value = psteps / (ms / 1e3)
    k_avg_s = (k_ms / max(k_n, 1)) / 1e3
    if grid and a.path == "plain":
        # dominant kernel: one streaming Euler step of every particle per launch
        nbytes = FHN_BYTES_PER_NODE_STEP * M * N * nodes
        achieved = nbytes / k_avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "k_grid_stream_step", "algorithmic_bytes_per_launch": nbytes}
    else:
        # dominant kernel: S Euler steps of every particle per launch, VALU-bound
        per = FHN_SLOTS_PER_NODE_STEP * nodes if grid else L63_SLOTS_PER_PARTICLE_STEP
        slots = per * M * N * S
        achieved = slots * FLOP_PER_SLOT / k_avg_s / 1e12
        peak = VALU_SLOTS_PER_S * FLOP_PER_SLOT / 1e12
        kname = {"fused": "k_grid_steps" if grid else "k_vec_prop_batched",
                 "graph": "interval graph", "plain": "k_vec_propagate"}[a.path]
        roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": None, "kernel": kname,
                    "algorithmic_slots_per_launch": slots}
    roofline["traffic"] = MEASURED_TRAFFIC_BYTES.get((spec["kind"], a.path, M, N))
    roofline.update({"kernel_avg_us": k_avg_s * 1e6, "launches": k_n,
                     "timed_intervals": f"every {PROF_EVERY}th of the timed region"})
    cpu = None
    if a.cpu_seconds > 0:
        cpu = cpu_baseline(spec, M, N, y.double().cpu().numpy(), a.cpu_seconds)
    acc = None
    if a.accuracy:
        del f
        torch.cuda.empty_cache()
        # the first ACCURACY_INTERVALS observations, whatever the warm-up
        acc = accuracy(pf, torch, spec, M, N, xt, y, min(T, ACCURACY_INTERVALS),
                       reference=a.workload.startswith("l63_sweep"))
    line = {
        "metric": "particle-steps/s", "value": value, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated truth and observations)",
        "config": {"workload": a.workload, "model": spec["kind"], "M": M, "N": N, "S": S,
                   "nodes_per_particle": nodes, "path": a.path, "wall_s": wall},
        "roofline": roofline, "cpu_baseline": cpu, "accuracy": acc,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
