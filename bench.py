"""Benchmark: particle-steps/s of the independent-ensemble bootstrap filter on
one MI355X.

A step is one observation interval of the whole hot path (S Euler-Maruyama
steps of every particle, weighting, normalisation, multinomial resampling,
gather and the ensemble estimate) over one batch; the headline workload is
the Lorenz 63 time-error sweep split M = 256 filters x N = 4096 particles
(K = 2^20 particles, S = 40 Euler steps per interval).  Observations are
synthetic: the library's own truth simulator on the GPU.

Prints one JSON line: the headline throughput, the dominant kernel's
roofline (timed live with HIP events around its launches in every
PROF_EVERY-th timed interval), the FP64 oracle timed on a bounded sample on
the host cores, and -- with the default workload -- the other measurements
of the hot path in extra keys, each timed with the same warm-up and step
counts (they run before the headline, whose timed intervals then see the
device at its sustained clock):
  sweep         every split M x N of K = 2^20 (M = 1, 16, 256, 4096): time per
                interval, MSE against the truth and against a 64 x 2^20
                reference filter, C_ipf = 1/M + 1/N;
  fhn40_64x512  the FH-N 40 x 40 ensemble on the blocked path (all S steps per
                launch, VALU-bound) and on the streaming path (one Euler step
                per launch, HBM-bound), with the MSE of both;
  mix           the uneven 1024 + 32 tenant batch, graph-replayed under the
                autotuner's plan against the plain one-kernel-per-step path,
                with the MSE of both;
  learned       the learned proposal against the bootstrap filter on the same
                observations: time per interval at a stated equal MSE;
  paper_l63     the paper's own Lorenz 63 experiment (Sec. 4): ensembles of
                M = 20 filters against the centralised filter of K = M N,
                MSE at t = 200 against a J = 1e5 proxy over 100 runs;
  paper_fhn     the paper's FH-N network (Sec. 5): ensembles of M = 10
                bootstrap filters against the centralised filter, MSE per
                node and time per discrete step.
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
#   for 128 lanes per CU per clock, i.e. 7.86e13 issue slots/s (the published
#   157.3 TFLOP/s FP32 is this rate at 2 FLOP per FMA).  Work is counted in
#   full-rate issue slots: half-rate instructions (32x32-bit integer
#   multiply, v_mad_u64_u32, FP64 FMA, int->float conversion) take 2 slots,
#   transcendentals (log2, sqrt, sin, cos, exp) take 4, their issue rates
#   relative to a 32-bit FMA.  Beside the slot fraction the line reports the
#   slots the compiled kernel issues (hardware counters, below) and the pure
#   FP32 FLOP fraction of the model arithmetic against 157.3 TFLOP/s.
HBM_PEAK_GBS = 8000.0
VALU_SLOTS_PER_S = 256 * 128 * 2.4e9
FP32_PEAK_TFLOPS = 157.3

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

# intervals of the untimed accuracy passes
ACCURACY_INTERVALS = 220

# Lorenz 63 particle-step: 3 Philox calls per 4 steps, 1.5 Box-Muller pairs,
# drift (7) and the Euler update (2 FMAs per component).
L63_SLOTS_PER_PARTICLE_STEP = 0.75 * PHILOX_SLOTS + 1.5 * BOXMULLER_SLOTS + 7 + 6
# FP32 FLOP of the Lorenz model arithmetic per particle-step: the drift
# (s(x2 - x1), x1(r - x3) - x2, x1 x2 - b x3: 8) and x + h f + sd sqrt(h) z
# (2 FMAs per component: 12), random-number generation excluded.
L63_FP32_FLOP_PER_PARTICLE_STEP = 20.0
# FH-N node-step: one Philox call per 2 nodes, one Box-Muller pair, the
# 4-neighbour Laplacian (7), reaction and recovery drifts (8), 2 x 2 FMAs.
FHN_SLOTS_PER_NODE_STEP = 0.5 * PHILOX_SLOTS + BOXMULLER_SLOTS + 7 + 8 + 4
# FP32 FLOP of the FH-N model arithmetic per node-step: Laplacian (7 adds),
# reaction v(v - a)(1 - v) - w + D lap (7), recovery eps (v - gam w) (3),
# two updates x + h f + sd sqrt(h) z (2 FMAs each: 8).
FHN_FP32_FLOP_PER_NODE_STEP = 25.0
# Issued VALU work per unit from rocprofv3 counters of one launch
# (SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32, SQ_INSTS_VALU_INT64, x 64 lanes /
# units; profiles/valu_instruction_mix.md): instructions per unit, and slots
# = instructions + 3 per transcendental + 1 per 64-bit multiply-add.
L63_ISSUED = {"valu": 60.33, "trans": 6.00, "int64": 11.85}
FHN_ISSUED = {"valu": 55.93, "trans": 4.48, "int64": 8.50}
# 64 lanes per CU per clock: the basis of the plain instruction-issue fraction
VALU_LANE_OPS_64_PER_S = 256 * 64 * 2.4e9


def issued_slots(mix):
    return mix["valu"] + 3 * mix["trans"] + mix["int64"]


# FH-N streaming Euler step: every node's v and w read and written once.
FHN_BYTES_PER_NODE_STEP = 16.0

# Learned proposal: the MLP 22 -> 64 -> 64 -> 2 per node and Euler step,
# 2 (22*64 + 64*64 + 64*2) FLOP, against the dense bfloat16 MFMA peak.
MLP_FLOP_PER_NODE_STEP = 2.0 * (22 * 64 + 64 * 64 + 64 * 2)
BF16_MFMA_PEAK_TFLOPS = 2500.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch of a timed-type interval, i.e. one that reads
# through the ancestors; fetch scaled x2, write x1 by the same counters on a
# 1 GiB copy), recorded in profiles/hbm_counters.md for the kernels as they
# are now.
MEASURED_TRAFFIC_BYTES = {
    ("lorenz63", "fused", 256, 4096): (2 * 2368.0 + 16384) * 1024,
    ("fhn", "plain", 64, 512): (2 * 204859.5 + 409604.4) * 1024,
    ("fhn_paper", "fused", 10, 5000): (2 * 202242.7 + 421123.3) * 1024,
}

SWEEP = (("l63_sweep_M1", 1, 1 << 20), ("l63_sweep_M16", 16, 1 << 16),
         ("l63_sweep_M256", 256, 1 << 12), ("l63_sweep_M4096", 4096, 1 << 8))


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
    ap.add_argument("--extras", type=int, default=1,
                    help="1 (default workload only): add the sweep, FH-N, mix and learned "
                         "measurements to the line")
    a = ap.parse_args()
    a.warmup_given = a.warmup is not None
    if a.warmup is None:
        kind = pf_inputs.WORKLOADS[a.workload][0]
        a.warmup = (200 if a.workload.startswith("mix") else
                    500 if kind is pf_inputs.lorenz63 else 20)
    return a


# ------------------------------------------------------------ CPU oracle ----
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
    paper spreads filters over cores (each filter single-threaded); about
    target_s seconds of wall time on every core used."""
    import concurrent.futures as cf
    import oracle
    oracle.lib()
    cores = max(1, min(16, os.cpu_count() or 1))
    # calibrate with one interval of one filter
    per_filter_interval = max(_oracle_worker((spec, 1, 0, N, 1, y_host)), 1e-6)
    intervals = max(1, min(len(y_host), int(target_s / per_filter_interval)))
    n_filters = min(M, cores)
    jobs = [(spec, 1, f, N, intervals, y_host) for f in range(n_filters)]
    t0 = time.perf_counter()
    # one thread per filter: the oracle's C calls release the GIL
    with cf.ThreadPoolExecutor(n_filters) as pool:
        list(pool.map(_oracle_worker, jobs))
    wall = time.perf_counter() - t0
    steps = n_filters * intervals * N * spec["S"]
    return {"value": steps / wall, "unit": "particle-steps/s", "cores": n_filters,
            "wall_s": wall, "kind": "oracle",
            "sample": f"{n_filters} filters x N={N} x {intervals} intervals "
                      f"({steps:.3g} particle-steps, FP64, one filter per core)",
            # the calibration run: one filter's interval on one core
            "single_core_value": N * spec["S"] / per_filter_interval}


# ------------------------------------------------------------- helpers ------
def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed_intervals(torch, f, y, warmup, steps, graph=False, est=None, est_rows=0):
    """`warmup` untimed intervals, then `steps` timed ones with the dominant
    kernel's events on every PROF_EVERY-th; returns (ms, kernel ms, kernel
    launches, wall s).  With `est`, the ensemble estimate of every timed
    interval is copied to est[k] (float64 device rows of `est_rows`)."""
    import ctypes as C
    import paper_1407_8071_amd as pf
    for t in range(warmup):
        f.step(None if graph else y[t])
    torch.cuda.synchronize()
    f.read_profile()
    stream = torch.cuda.current_stream()
    e0, e1 = _events(torch)
    t0 = time.perf_counter()
    e0.record(stream)
    for k, t in enumerate(range(warmup, warmup + steps)):
        f.set_profiling(k % PROF_EVERY == 0)
        f.step(None if graph else y[t])
        if est is not None:
            pf._check(pf.lib().pf_estimate(f._ctx, C.c_void_p(est[k].data_ptr()), None, None,
                                           None, pf._stream(None)))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f.set_profiling(False)
    k_ms, k_n = f.read_profile()
    del est_rows
    return e0.elapsed_time(e1), k_ms, k_n, wall


def estimates(pf, torch, spec, M, N, y, T, flags=0, params=None):
    """Untimed: a fresh fused filter over y[0:T]; the ensemble estimate of
    every interval, [T][dx] float64 on the device."""
    import ctypes as C
    f = pf.ParticleFilter([spec], [(0, M, N, 1, flags)], fused=True)
    if params is not None:
        f.set_proposal(0, params)
    est = torch.empty((T, spec["dx"]), dtype=torch.float64, device="cuda")
    for t in range(T):
        f.step(y[t])
        pf._check(pf.lib().pf_estimate(f._ctx, C.c_void_p(est[t].data_ptr()), None, None, None,
                                       pf._stream(None)))
    torch.cuda.synchronize()
    f.close()
    return est


def valu_roofline(kernel, slots, flop, k_avg_s, launches, units=None, issued=None):
    """VALU issue-slot fraction of a kernel against 7.86e13 slots/s, with the
    pure FP32 FLOP fraction of its model arithmetic beside it; with the
    counter-measured instruction mix of the kernel (per unit) also the slots
    it issues and its instruction count against 64 lanes per CU per clock."""
    achieved = slots / k_avg_s / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    tflops = flop / k_avg_s / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T VALU-slots/s",
         "frac": achieved / peak, "traffic": None, "kernel": kernel,
         "algorithmic_slots_per_launch": slots,
         "fp32_flop_per_launch": flop, "fp32_tflops": tflops,
         "fp32_flop_frac": tflops / FP32_PEAK_TFLOPS,
         "kernel_avg_us": k_avg_s * 1e6, "launches": launches,
         "timed_intervals": f"every {PROF_EVERY}th of the timed region"}
    if issued is not None and units:
        s_issued = issued_slots(issued) * units
        r["issued_slots_per_launch_counters"] = s_issued
        r["issued_slot_frac"] = s_issued / k_avg_s / VALU_SLOTS_PER_S
        r["valu_instr_frac_64_lanes"] = issued["valu"] * units / k_avg_s / VALU_LANE_OPS_64_PER_S
    return r


# ------------------------------------------------------ Lorenz sweep --------
def sweep_leg(pf, torch, a, spec, xt, y, head):
    """Every split of K = 2^20: time per interval (same warm-up and steps as
    the headline), then an untimed accuracy pass over ACCURACY_INTERVALS
    against the truth and against 64 filters x 2^20 particles."""
    T = ACCURACY_INTERVALS
    truth = xt[1:T + 1].double()
    ref = estimates(pf, torch, spec, 64, 1 << 20, y, T)
    out = {"reference": "64 x 2^20 fused filter on the same observations",
           "accuracy_intervals": T,
           "reference_mse_vs_truth": torch.mean((ref - truth) ** 2).item(), "splits": []}
    for name, M, N in SWEEP:
        if name == a.workload and head is not None:
            ms, k_ms, k_n = head
        else:
            f = pf.ParticleFilter([spec], [(0, M, N, 1)], fused=True)
            ms, k_ms, k_n, _ = timed_intervals(torch, f, y, a.warmup, a.steps)
            f.close()
        est = estimates(pf, torch, spec, M, N, y, T)
        out["splits"].append({
            "M": M, "N": N, "ms_per_interval": ms / a.steps,
            "particle_steps_per_s": M * N * spec["S"] * a.steps / (ms / 1e3),
            "propagation_kernel_avg_us": k_ms / max(k_n, 1) * 1e3,
            "mse_vs_truth": torch.mean((est - truth) ** 2).item(),
            "mse_vs_reference": torch.mean((est - ref) ** 2).item(),
            "c_ipf": 1.0 / M + 1.0 / N})
        del est
    del ref
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------ FH-N 40 x 40 --------
def fhn_leg(pf, torch, a):
    """FH-N 40 x 40, M = 64 x N = 512: the blocked fused path and the plain
    streaming path on the same observations; the streaming step against the
    HBM roofline, the blocked stepping against the VALU roofline; MSE of the
    v nodes against the truth over the timed intervals of both."""
    spec = pf_inputs.fhn(40)
    M, N = 64, 512
    nn = spec["J"] ** 2
    T = a.warmup + a.steps
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    xt, y = sim.simulate(0, 1, T)
    sim.close()
    truth = xt[1 + a.warmup:1 + T, :nn].double()
    out = {"J": 40, "M": M, "N": N, "S": spec["S"]}
    for path in ("fused", "plain"):
        f = pf.ParticleFilter([spec], [(0, M, N, 1)], fused=(path == "fused"))
        est = torch.empty((a.steps, spec["dx"]), dtype=torch.float64, device="cuda")
        ms, k_ms, k_n, _ = timed_intervals(torch, f, y, a.warmup, a.steps, est=est)
        f.close()
        k_avg_s = k_ms / max(k_n, 1) / 1e3
        r = {"ms_per_interval": ms / a.steps,
             "particle_steps_per_s": M * N * spec["S"] * a.steps / (ms / 1e3),
             "node_steps_per_s": M * N * nn * spec["S"] * a.steps / (ms / 1e3),
             "mse_v_vs_truth": torch.mean((est[:, :nn] - truth) ** 2).item()}
        if path == "fused":
            units = M * N * nn * spec["S"]
            r["roofline"] = valu_roofline("k_grid_steps (all S steps, plane in LDS)",
                                          FHN_SLOTS_PER_NODE_STEP * units,
                                          FHN_FP32_FLOP_PER_NODE_STEP * units, k_avg_s, k_n,
                                          units, FHN_ISSUED)
            out["blocked"] = r
        else:
            nbytes = FHN_BYTES_PER_NODE_STEP * M * N * nn
            gbs = nbytes / k_avg_s / 1e9
            r["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                             "traffic": MEASURED_TRAFFIC_BYTES.get(("fhn", "plain", M, N)),
                             "kernel": "k_grid_stream_step (one Euler step per launch)",
                             "algorithmic_bytes_per_launch": nbytes,
                             "kernel_avg_us": k_avg_s * 1e6, "launches": k_n,
                             "timed_intervals": f"every {PROF_EVERY}th of the timed region"}
            out["streaming"] = r
        del est
        torch.cuda.empty_cache()
    out["blocked_speedup_vs_streaming"] = (out["streaming"]["ms_per_interval"] /
                                           out["blocked"]["ms_per_interval"])
    return out


# ------------------------------------------------------ uneven mix ----------
def mix_leg(pf, torch, a, n_compare=4):
    """The uneven serving mix: 1024 Lorenz 63 tenants with N log-uniform in
    [64, 8192] and 32 FH-N 20 x 20 tenants with N in {128, 256, 512}, each an
    ensemble of one filter with its own seed and observations; one
    graph-replayed fused interval per observation under the autotuner's plan,
    against the plain path (one kernel per method step and tenant).  Both
    paths compute the same filter: their MSE against the truth over the
    first n_compare intervals is reported side by side."""
    n_l, n_f = pf_inputs.mixed_batch(1)
    specs = [pf_inputs.lorenz63(), pf_inputs.fhn(20)]
    ens = [(0, 1, n, 1000 + i) for i, n in enumerate(n_l)] + \
          [(1, 1, n, 5000 + i) for i, n in enumerate(n_f)]
    T = max(a.warmup + a.steps, n_compare + 3)
    sim = pf.ParticleFilter(specs, [(0, 1, 1, 1), (1, 1, 1, 1)], fused=True)
    ys, xs = [], []
    for (mi, _, _, seed) in ens:
        x, y = sim.simulate(mi, seed, T)
        ys.append(y)
        xs.append(x)
    sim.close()
    y_all = torch.cat(ys, dim=1).contiguous()
    truth = torch.cat([x for x in xs], dim=1).double()    # [T+1][sum dx]
    del ys, xs
    psteps = sum(n * specs[mi]["S"] for (mi, _, n, _) in ens)
    l63_ps = sum(n * 40 for n in n_l)
    fhn_ps = sum(n * 20 for n in n_f)

    def track(f, graph):
        est = torch.empty((n_compare, truth.shape[1]), dtype=torch.float64, device="cuda")
        for t in range(n_compare):
            f.step(None if graph else y_all[t])
            est[t] = f.estimate()[0]
        return torch.mean((est - truth[1:n_compare + 1]) ** 2).item(), est

    # autotuned plan, graph replay of the staged observations
    f = pf.ParticleFilter(specs, ens, graph=True)
    t0 = time.perf_counter()
    tuning = f.autotune(y_all[0], reps=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    f.set_observations(y_all)
    mse_graph, est_graph = track(f, True)
    f.close()
    f = pf.ParticleFilter(specs, ens, graph=True)
    f.set_tuning(tuning)
    f.set_observations(y_all)
    ms, _, _, wall = timed_intervals(torch, f, y_all, a.warmup, a.steps, graph=True)
    f.close()
    # the propagation kernels with events, on a directly launched context
    g = pf.ParticleFilter(specs, ens, fused=True)
    g.set_tuning(tuning)
    nprof = max(1, min(20, a.steps))
    _, k_ms, k_n, _ = timed_intervals(torch, g, y_all, min(3, a.warmup), nprof)
    g.close()
    slots = (L63_SLOTS_PER_PARTICLE_STEP * l63_ps + FHN_SLOTS_PER_NODE_STEP * 400 * fhn_ps)
    flop = (L63_FP32_FLOP_PER_PARTICLE_STEP * l63_ps + FHN_FP32_FLOP_PER_NODE_STEP * 400 * fhn_ps)
    # profiling brackets every PROF_EVERY-th interval's propagation launches
    prof_intervals = (nprof + PROF_EVERY - 1) // PROF_EVERY
    rl = valu_roofline("propagation kernels (Lorenz tiles + batched FH-N steps), summed",
                       slots, flop, k_ms / 1e3 / prof_intervals, k_n)
    rl["kernel_ms_per_interval"] = k_ms / prof_intervals
    # the plain path: same filter, one kernel per method step and tenant
    pl = pf.ParticleFilter(specs, ens, fused=False)
    mse_plain, est_plain = track(pl, False)
    n_plain = 3
    e0, e1 = _events(torch)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for t in range(n_compare, n_compare + n_plain):
        pl.step(y_all[t])
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / n_plain
    pl.close()
    return {"tenants_l63": len(n_l), "tenants_fhn20": len(n_f),
            "particles_l63": int(sum(n_l)), "particles_fhn": int(sum(n_f)),
            "particle_steps_per_interval": psteps, "tuning": tuning, "tune_s": tune_s,
            "graph_ms_per_interval": ms / a.steps,
            "graph_particle_steps_per_s": psteps * a.steps / (ms / 1e3),
            "plain_ms_per_interval": plain_ms,
            "graph_speedup_vs_plain": plain_ms / (ms / a.steps),
            "equal_mse": {"intervals": n_compare, "mse_vs_truth_graph": mse_graph,
                          "mse_vs_truth_plain": mse_plain,
                          "max_abs_estimate_difference":
                              torch.max(torch.abs(est_graph - est_plain)).item()},
            "roofline": rl}


# ------------------------------------------------------ the paper's Lorenz --
def paper_l63_leg(pf, torch, a):
    """The paper's own Lorenz experiment (Sec. 4.2-4.3): one observation record
    of 200 intervals (x1 every 100 Euler steps), the ensemble of M = 20
    independent filters of N particles and the centralised filter of K = M N
    particles, 100 runs each (independent seeds, the same observations) for
    every N; per run the squared error of the posterior-mean estimate at
    t = 200 against the estimate of one filter of J = 1e5 particles (the
    paper's proxy), reported as the mean and the variance over the runs.  The
    100 runs of a configuration are 100 ensembles of one graph-replayed
    context; the time per run is that batch's time / 100, and the time of
    one run alone is measured too."""
    cfg = pf_inputs.PAPER_L63
    spec = pf_inputs.lorenz63_paper()
    T, R, M = cfg["T"], cfg["runs"], cfg["M"]
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    xt, y = sim.simulate(0, 1, T)
    sim.close()
    stream = torch.cuda.current_stream()

    def run(ens, timed=True):
        """All intervals of a context of ensembles `ens` on the shared
        observations; returns (ms, estimates at t = T [n_ens][3])."""
        f = pf.ParticleFilter([spec], ens, graph=True)
        f.set_observations(y.repeat(1, len(ens)).contiguous())
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record(stream)
        for _ in range(T):
            f.step()
        e1.record(stream)
        est = f.estimate()[0].view(len(ens), 3).clone()
        torch.cuda.synchronize()
        f.close()
        return e0.elapsed_time(e1), est

    _, proxy = run([(0, 1, cfg["proxy_J"], 99)])
    proxy = proxy[0]
    rows = []
    for N in cfg["Ns"]:
        r = {"N": N, "K": M * N}
        for name, ens, single in (
                ("ensemble", [(0, M, N, 1000 + i) for i in range(R)], (0, M, N, 1000)),
                ("centralised", [(0, 1, M * N, 5000 + i) for i in range(R)], (0, 1, M * N, 5000))):
            ms, est = run(ens)
            err = torch.sum((est - proxy) ** 2, dim=1)     # squared error per run
            ms1, _ = run([single])
            r[name] = {"mse_mean": err.mean().item(), "mse_var": err.var().item(),
                       "ms_per_run_batched": ms / R, "ms_per_run_alone": ms1,
                       "particle_steps_per_s_batched":
                           R * M * N * spec["S"] * T / (ms / 1e3)}
        rows.append(r)
    return {"model": "Lorenz 63, x1 observed every 100 steps (var 1/2), unit diffusion, "
                     "prior N(x*, 10 I)", "T": T, "M": M, "runs": R,
            "proxy": "one bootstrap filter of J = %d particles" % cfg["proxy_J"],
            "error": "squared Euclidean error of E[X_t | y_1:t] at t = T against the proxy "
                     "(mean and variance over the runs)",
            "proxy_estimate": proxy.tolist(), "truth_at_T": xt[T].tolist(), "rows": rows}


def paper_fhn_leg(pf, torch, a, datasets=5, T=300):
    """The paper's FH-N network experiment (Sec. 5.3) with the auxiliary
    filter the paper runs and with the bootstrap filter: ensembles of M = 10
    independent filters of N particles against
    the centralised filter of K = M N particles (K <= 8192, the per-filter
    resampler's limit), on `datasets` independent truth records of T
    discrete steps (one observation per step); the MSE per node of the U
    estimate against the truth over the steps after the first 50, averaged
    over the records, and the time per discrete step (all records' filters
    batched in one graph-replayed context, and one filter ensemble alone)."""
    spec = pf_inputs.fhn_paper(32)
    nn = spec["J"] ** 2
    M = pf_inputs.PAPER_FHN["M"]
    skip = 50
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    recs = [sim.simulate(0, 900 + r, T) for r in range(datasets)]
    sim.close()
    truth = torch.stack([x[1:, :nn] for x, _ in recs]).double()    # [R][T][nn]
    y_all = torch.cat([y for _, y in recs], dim=1).contiguous()
    stream = torch.cuda.current_stream()

    import ctypes as C

    def run(Mf, N, flags=0):
        """(ms per step of the timed pass, MSE of an untimed pass that
        copies the ensemble estimates out at every step)."""
        ens = [(0, Mf, N, 70 + r, flags) for r in range(datasets)]
        f = pf.ParticleFilter([spec], ens, graph=True)
        f.set_observations(y_all)
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record(stream)
        for t in range(T):
            f.step()
        e1.record(stream)
        torch.cuda.synchronize()
        f.close()
        ms = e0.elapsed_time(e1) / T
        f = pf.ParticleFilter([spec], ens, graph=True)
        f.set_observations(y_all)
        est = torch.empty((T, datasets, spec["dx"]), dtype=torch.float64, device="cuda")
        for t in range(T):
            f.step()
            pf._check(pf.lib().pf_estimate(f._ctx, C.c_void_p(est[t].data_ptr()), None, None,
                                           None, pf._stream(None)))
        torch.cuda.synchronize()
        f.close()
        err = (est[skip:, :, :nn].permute(1, 0, 2) - truth[:, skip:]) ** 2
        return ms, err.mean().item()

    rows = []
    for N in pf_inputs.PAPER_FHN["Ns"]:
        r = {"N": N, "K": M * N}
        for name, flags in (("bootstrap", 0), ("auxiliary", pf.ENS_AUXILIARY)):
            ms_e, mse_e = run(M, N, flags)
            r[name + "_ensemble"] = {"mse_per_node": mse_e, "ms_per_step_all_records": ms_e}
            if M * N <= 8192:
                ms_c, mse_c = run(1, M * N, flags)
                r[name + "_centralised"] = {"mse_per_node": mse_c,
                                            "ms_per_step_all_records": ms_c}
        rows.append(r)
    return {"model": "the paper's FH-N network (32 x 32, stimuli, forcing)",
            "filters": "bootstrap and auxiliary (the paper's), ensembles of M and centralised",
            "M": M, "records": datasets, "steps": T, "mse_after_step": skip, "rows": rows}


# ------------------------------------------------------ learned proposal ----
def train_proposal(pf, torch, spec):
    tc = pf_inputs.LEARNED_TRAINING
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
    return p, {"trajectories": tc["n_runs"] * tc["run_len"], "adam_steps": n_steps,
               "rows_per_step": 16 * tc["batch_tiles"], "data_s": t_data, "train_s": t_train}


LEARNED_NS = (32, 64, 128)
BOOTSTRAP_NS = (128, 512, 2048)
LEARNED_EVAL_INTERVALS = 100
LEARNED_SKIP = 20


def learned_leg(pf, torch, a, p=None, training=None):
    """FH-N 40 x 40, M = 64 filters: the learned proposal at N in LEARNED_NS
    and the bootstrap filter at N in BOOTSTRAP_NS on the same GPU-simulated
    observations.  Every filter runs LEARNED_SKIP + LEARNED_EVAL_INTERVALS
    intervals; the MSE of the v nodes against the truth is taken over the
    last LEARNED_EVAL_INTERVALS (after the wave's launch transient), and the
    time per interval over the last `steps` of them.  Equal MSE: the smallest
    learned N whose MSE does not exceed the bootstrap filter's at N = 512
    (and at N = 2048), and the ratio of their times."""
    import ctypes as C
    spec = pf_inputs.fhn(40)
    M = 64
    nn = spec["J"] ** 2
    if p is None:
        p, training = train_proposal(pf, torch, spec)
    T = LEARNED_SKIP + max(LEARNED_EVAL_INTERVALS, a.steps)
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    xt, y = sim.simulate(0, 1, T)
    sim.close()
    truth = xt[1:T + 1, :nn].double()
    runs = [("learned", n, pf.ENS_LEARNED) for n in LEARNED_NS] + \
           [("bootstrap", n, 0) for n in BOOTSTRAP_NS]
    res = []
    for kind, N, flags in runs:
        f = pf.ParticleFilter([spec], [(0, M, N, 1, flags)], fused=True)
        if flags:
            f.set_proposal(0, p)
        est = torch.empty((T, spec["dx"]), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        e0, e1 = _events(torch)
        t_from = T - a.steps
        for t in range(T):
            if t == t_from:
                torch.cuda.synchronize()
                f.read_profile()
                e0.record(stream)
            if t >= t_from:
                f.set_profiling((t - t_from) % PROF_EVERY == 0)
            f.step(y[t])
            pf._check(pf.lib().pf_estimate(f._ctx, C.c_void_p(est[t].data_ptr()), None, None,
                                           None, pf._stream(None)))
        e1.record(stream)
        torch.cuda.synchronize()
        f.set_profiling(False)
        k_ms, k_n = f.read_profile()
        f.close()
        ms = e0.elapsed_time(e1) / a.steps
        mse = torch.mean((est[LEARNED_SKIP:, :nn] - truth[LEARNED_SKIP:]) ** 2).item()
        res.append({"proposal": kind, "M": M, "N": N, "ms_per_interval": ms, "mse_v": mse,
                    "particle_steps_per_s": M * N * spec["S"] / (ms / 1e3),
                    "kernel_avg_us": k_ms / max(k_n, 1) * 1e3, "kernel_launches": k_n})
        del est
        torch.cuda.empty_cache()
    learned = [r for r in res if r["proposal"] == "learned"]
    boot = {r["N"]: r for r in res if r["proposal"] == "bootstrap"}
    equal = []
    for nb in (512, 2048):
        b = boot[nb]
        ok = [r for r in learned if r["mse_v"] <= b["mse_v"]]
        if ok:
            r = min(ok, key=lambda r: r["N"])
            equal.append({"bootstrap_N": nb, "bootstrap_mse_v": b["mse_v"],
                          "bootstrap_ms_per_interval": b["ms_per_interval"],
                          "learned_N": r["N"], "learned_mse_v": r["mse_v"],
                          "learned_ms_per_interval": r["ms_per_interval"],
                          "speedup": b["ms_per_interval"] / r["ms_per_interval"]})
        else:
            equal.append({"bootstrap_N": nb, "bootstrap_mse_v": b["mse_v"],
                          "learned_N": None,
                          "note": "no learned N in %s reaches this MSE" % (LEARNED_NS,)})
    L = max(learned, key=lambda r: r["N"])
    k_avg_s = L["kernel_avg_us"] / 1e6
    flop = MLP_FLOP_PER_NODE_STEP * nn * spec["S"] * M * L["N"]
    achieved = flop / k_avg_s / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                "kernel": "k_grid_steps_learned (N = %d)" % L["N"],
                "algorithmic_flop_per_launch": flop, "kernel_avg_us": L["kernel_avg_us"],
                "launches": L["kernel_launches"],
                "timed_intervals": f"every {PROF_EVERY}th of the timed region"}
    return {"J": 40, "M": M, "mse_intervals": LEARNED_EVAL_INTERVALS,
            "skipped_intervals": LEARNED_SKIP, "network_inputs": 22,
            "runs": res, "equal_mse": equal, "training": training, "roofline": roofline}, p


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
    """The learned workload as the headline: the learned filter at N = 128
    is the line's value, the bootstrap runs and the equal-MSE comparison
    are extra keys."""
    import torch
    import paper_1407_8071_amd as pf
    torch.cuda.set_device(0)
    out, p = learned_leg(pf, torch, a)
    L = [r for r in out["runs"] if r["proposal"] == "learned" and r["N"] == 128][0]
    spec = pf_inputs.fhn(40)
    cpu = None
    if a.cpu_seconds > 0:
        sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
        _, y = sim.simulate(0, 1, 1)
        sim.close()
        cpu = cpu_baseline_learned(spec, p.double().cpu().numpy(), y.double().cpu().numpy(),
                                   a.cpu_seconds)
    line = {
        "metric": "particle-steps/s", "value": L["particle_steps_per_s"],
        "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": LEARNED_SKIP,
        "ms_per_step": L["ms_per_interval"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 MFMA network, f32 filter",
        "data": "synthetic (GPU-simulated truth and observations; model-simulated training paths)",
        "config": {"workload": a.workload, "model": "fhn", "J": 40, "M": 64, "N": 128,
                   "S": spec["S"], "path": "fused", "network_inputs": 22},
        "roofline": out.pop("roofline"), "cpu_baseline": cpu, "learned": out,
    }
    print(json.dumps(line))


def mix_main(a):
    import torch
    import paper_1407_8071_amd as pf
    torch.cuda.set_device(0)
    out = mix_leg(pf, torch, a)
    line = {
        "metric": "particle-steps/s", "value": out["graph_particle_steps_per_s"],
        "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": out["graph_ms_per_interval"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated truth and observations per tenant)",
        "config": {"workload": a.workload, "path": "graph"},
        "roofline": out.pop("roofline"), "cpu_baseline": None, "mix": out,
    }
    print(json.dumps(line))


def paper_main(a):
    """The paper's Lorenz experiment as the headline: the value is the
    batched ensemble runs' particle-steps/s at the largest N."""
    import torch
    import paper_1407_8071_amd as pf
    torch.cuda.set_device(0)
    out = paper_l63_leg(pf, torch, a)
    last = out["rows"][-1]["ensemble"]
    cfg = pf_inputs.PAPER_L63
    line = {
        "metric": "particle-steps/s", "value": last["particle_steps_per_s_batched"],
        "unit": "particle-steps/s", "n_gpus": 1, "steps": cfg["T"], "warmup": 0,
        "ms_per_step": last["ms_per_run_batched"] / cfg["T"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated truth and observations)",
        "config": {"workload": a.workload, "M": cfg["M"], "N": cfg["Ns"][-1],
                   "runs": cfg["runs"], "path": "graph"},
        "roofline": None, "cpu_baseline": None, "paper_l63": out,
    }
    print(json.dumps(line))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the ensemble would shard by whole filters, one group of filters per GPU)",
              file=sys.stderr)
        sys.exit(2)
    if a.workload == "fhn40_learned_64x128":
        learned_main(a)
        return
    if a.workload == "mix_l63x1024_fhn20x32":
        mix_main(a)
        return
    if a.workload == "l63_paper":
        paper_main(a)
        return
    import torch
    import paper_1407_8071_amd as pf

    factory, M, N, T_cfg = pf_inputs.WORKLOADS[a.workload]
    spec = factory()
    grid = spec["kind"] in ("fhn", "fhn_paper")
    torch.cuda.set_device(0)
    graph = a.path == "graph"
    T = a.warmup + a.steps
    sim = pf.ParticleFilter([spec], [(0, 1, 1, 1)], fused=True)
    xt, y = sim.simulate(0, 1, max(T, ACCURACY_INTERVALS))
    sim.close()
    torch.cuda.synchronize()
    extras = {}
    sweep = a.workload.startswith("l63_sweep")
    if sweep and a.extras and a.path == "fused":
        # the other measurements of the line first: the headline's timed
        # intervals then see the device at its sustained clock (the first
        # few hundred intervals of a cold device measured ~6% slower)
        t0 = time.perf_counter()
        extras["fhn40_64x512"] = fhn_leg(pf, torch, a)
        extras["mix"] = mix_leg(pf, torch, a)
        extras["learned"], _ = learned_leg(pf, torch, a)
        extras["paper_l63"] = paper_l63_leg(pf, torch, a)
        extras["paper_fhn"] = paper_fhn_leg(pf, torch, a)
        extras["sweep"] = sweep_leg(pf, torch, a, spec, xt, y, None)
        extras["extras_wall_s"] = time.perf_counter() - t0
        torch.cuda.empty_cache()
    f = pf.ParticleFilter([spec], [(0, M, N, 1)], fused=(a.path == "fused"), graph=graph)
    if graph:
        f.set_observations(y)
    ms, k_ms, k_n, wall = timed_intervals(torch, f, y, a.warmup, a.steps, graph=graph)
    f.sync()
    est = f.estimate()[0].cpu().numpy()
    assert np.all(np.isfinite(est)), "non-finite estimate"
    f.close()

    S = spec["S"]
    nodes = spec["J"] ** 2 if grid else 1
    value = M * N * S * a.steps / (ms / 1e3)
    k_avg_s = (k_ms / max(k_n, 1)) / 1e3
    if spec["kind"] == "fhn_paper":
        # dominant kernel: every particle's interval with the planes in LDS;
        # its HBM bytes are one read and one write of each particle's state
        nbytes = 2.0 * 4 * spec["dx"] * M * N
        achieved = nbytes / k_avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "k_fhnp_steps", "algorithmic_bytes_per_launch": nbytes,
                    "kernel_avg_us": k_avg_s * 1e6, "launches": k_n,
                    "timed_intervals": f"every {PROF_EVERY}th of the timed region"}
    elif grid and a.path == "plain":
        # dominant kernel: one streaming Euler step of every particle per launch
        nbytes = FHN_BYTES_PER_NODE_STEP * M * N * nodes
        achieved = nbytes / k_avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "k_grid_stream_step", "algorithmic_bytes_per_launch": nbytes,
                    "kernel_avg_us": k_avg_s * 1e6, "launches": k_n,
                    "timed_intervals": f"every {PROF_EVERY}th of the timed region"}
    else:
        # dominant kernel: S Euler steps of every particle per launch, VALU-bound
        units = M * N * S * nodes
        per_slots = FHN_SLOTS_PER_NODE_STEP if grid else L63_SLOTS_PER_PARTICLE_STEP
        per_flop = FHN_FP32_FLOP_PER_NODE_STEP if grid else L63_FP32_FLOP_PER_PARTICLE_STEP
        kname = {"fused": "k_grid_steps" if grid else "k_vec_prop_batched",
                 "graph": "interval graph", "plain": "k_vec_propagate"}[a.path]
        issued = (FHN_ISSUED if grid else L63_ISSUED) if a.path == "fused" else None
        roofline = valu_roofline(kname, per_slots * units, per_flop * units, k_avg_s, k_n,
                                 units, issued)
    roofline["traffic"] = MEASURED_TRAFFIC_BYTES.get((spec["kind"], a.path, M, N))
    cpu = None
    if a.cpu_seconds > 0:
        cpu = cpu_baseline(spec, M, N, y.double().cpu().numpy(), a.cpu_seconds)
    line = {
        "metric": "particle-steps/s", "value": value, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated truth and observations)",
        "config": {"workload": a.workload, "model": spec["kind"], "M": M, "N": N, "S": S,
                   "nodes_per_particle": nodes, "path": a.path, "wall_s": wall},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    line.update(extras)
    if not extras and a.accuracy:
        torch.cuda.empty_cache()
        Ta = ACCURACY_INTERVALS
        comps = nodes if grid else spec["dx"]
        e = estimates(pf, torch, spec, M, N, y, Ta)
        truth = xt[1:Ta + 1, :comps].double()
        line["accuracy"] = {"intervals": Ta, "mse_vs_truth":
                            torch.mean((e[:, :comps] - truth) ** 2).item(),
                            "c_ipf": 1.0 / M + 1.0 / N}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
