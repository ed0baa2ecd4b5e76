"""Benchmark: particle-steps/s of the independent-ensemble bootstrap filter on
one MI355X.

A step is one observation interval of the whole hot path (S Euler-Maruyama
steps of every particle, weighting, normalisation, multinomial resampling,
gather and the ensemble estimate) over one batch; the default workload is the
Lorenz 63 time-error sweep split M = 256 filters x N = 4096 particles
(K = 2^20 particles, S = 40 Euler steps per interval).  Observations are
synthetic: the library's own truth simulator on the GPU.

Prints one JSON line with the throughput, the dominant kernel's roofline
(timed live with HIP events around each of its launches) and the FP64 oracle
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
# Roofline constants (MI355X: 256 CUs x 64 lanes x 2.4 GHz).
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9   # full-rate VALU lane-operations per second
HBM_PEAK_GBS = 8000.0

# Algorithmic VALU work of one Lorenz 63 particle-step, in full-rate lane-op
# slots (a quarter-rate instruction -- 32-bit integer multiply, transcendental
# -- occupies four):
#   Philox4x32-10, 3 calls per 4 steps: 10 rounds x (2 wide products x 4
#     + 2 three-input XORs) = 100 per call                        -> 75.0
#   Box-Muller, 1.5 pairs per step: 2 x 3 for the uniforms, log2, sqrt,
#     sin, cos (4 each), 3 multiplies                              -> 37.5
#   drift (8) and Euler update (6 FMAs)                            -> 14.0
L63_SLOTS_PER_PARTICLE_STEP = 126.5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="l63_sweep_M256", choices=sorted(pf_inputs.WORKLOADS))
    ap.add_argument("--path", default="plain", choices=["plain", "fused"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0 disables it)")
    return ap.parse_args()


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
            "kind": "oracle",
            "sample": f"{n_filters} filters x N={N} x {intervals} intervals "
                      f"({steps:.3g} particle-steps, FP64, one filter per core)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the ensemble shards by whole filters, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1407_8071_amd as pf

    factory, M, N, T_cfg = pf_inputs.WORKLOADS[a.workload]
    spec = factory()
    if spec["kind"] != "lorenz63":
        raise SystemExit("this bench times the Lorenz workloads")
    torch.cuda.set_device(0)
    f = pf.ParticleFilter([spec], [(0, M, N, 1)], fused=(a.path == "fused"))
    T = a.warmup + a.steps
    _, y = f.simulate(0, 1, T)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    for t in range(a.warmup):
        f.step(y[t])
    torch.cuda.synchronize()
    f.read_profile()
    f.set_profiling(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for t in range(a.warmup, T):
        f.step(y[t])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    f.set_profiling(False)
    k_ms, k_n = f.read_profile()
    est = f.estimate()[0].cpu().numpy()
    assert np.all(np.isfinite(est)), "non-finite estimate"

    S = spec["S"]
    psteps = M * N * S * a.steps
    ms_per_step = ms / a.steps
    value = psteps / (ms / 1e3)
    k_avg_s = (k_ms / max(k_n, 1)) / 1e3
    slots = L63_SLOTS_PER_PARTICLE_STEP * M * N * S
    achieved = slots / k_avg_s
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_SLOTS_PER_S / 1e12,
                "unit": "TOP/s", "frac": achieved / VALU_SLOTS_PER_S, "traffic": None,
                "kernel": "k_vec_propagate" if a.path == "plain" else "k_fused_interval",
                "kernel_avg_us": k_avg_s * 1e6, "launches": k_n}
    cpu = None
    if a.cpu_seconds > 0:
        cpu = cpu_baseline(spec, M, N, y.double().cpu().numpy(), a.cpu_seconds)
    line = {
        "metric": "particle-steps/s", "value": value, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated truth and observations)",
        "config": {"workload": a.workload, "model": "lorenz63", "M": M, "N": N, "S": S,
                   "path": a.path, "wall_s": wall},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
