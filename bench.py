"""Benchmark: batched persistent rollouts of uneven stations on one MI355X.

Workload (the uneven-batching configuration): 65,536 stations whose port counts
are drawn from {8, 16, 32, 64, 128} with probabilities {.3, .3, .2, .15, .05},
capacity trees 1-3 levels deep (fan-out 4, limits 0.7x the children's maxima),
288 five-minute steps, Philox random levels, every per-step record written
(observations, levels, rewards, done flags).  One bench "step" = one rollout of
all stations over all 288 steps in one persistent, graph-replayed launch.

Prints one JSON line: env-steps/s, the HBM roofline of the rollout kernel, the
plain one-launch-per-step form on the same GPU, and the FP64 oracle on the
host's cores as the CPU baseline.
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

HBM_PEAK_GBS = 8000.0
N_ENVS = 65536
T = 288


def record_bytes(n_ports: np.ndarray) -> np.ndarray:
    """Bytes of one FULL record per env-step: obs (6N+4) f32, N levels, reward f32, done u8."""
    return 4 * (6 * n_ports + 4) + n_ports + 4 + 1


def state_bytes(n_ports: np.ndarray) -> np.ndarray:
    """Per env: 1 - SoC (f64), 1 - target, capacity, last power (f32) and dwell (i16)
    per port, plus the f64 return."""
    return 22 * n_ports + 8


def measured_traffic():
    """HBM bytes of one rollout from the committed counter profile, if it was taken
    on the current kernel source (None otherwise)."""
    import hashlib
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "k_rollout_traffic.json")))
        src = open(os.path.join(ROOT, "paper_2507_01522_amd", "csrc", "cx_kernels.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest()[:16] != prof.get("kernel_sha256_prefix"):
        return None
    return float(prof["traffic_bytes"])


def workload():
    import workloads as W
    classes = W.mixture_classes()
    ec_full = W.mixture_env_classes(N_ENVS, seed=1003)
    specs, ec = W.compact_classes(classes, ec_full)
    return specs, ec


def cpu_baseline(specs, ec, seed):
    """The FP64 oracle on a bounded, evenly spaced sample of the same stations."""
    from oracle import oracle as o
    stride = 8
    ids = np.arange(0, len(ec), stride, dtype=np.int64)
    classes = [o.OracleClass(s) for s in specs]
    bs = o.BatchState(classes, ec[ids], env_ids=ids)
    threads = max(1, min(16, os.cpu_count() or 1))
    chunk = 16
    t0 = time.perf_counter()
    used = 1
    for _ in range(T // chunk):
        out = o.rollout(bs, seed, chunk, n_threads=threads)
        used = out["threads"]
    dt = time.perf_counter() - t0
    return {"value": len(ids) * T / dt, "unit": "env-steps/s", "cores": int(used), "kind": "oracle",
            "sample": f"{len(ids)} of {len(ec)} stations (every {stride}th), all {T} steps, FP64, "
                      f"all outputs, {used} threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-step comparison")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 2 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the rollout has no cross-GPU work; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2507_01522_amd as cx

    if args.calib_copy:
        src = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    seed = 3
    specs, ec = workload()
    n_ports = np.array([s.n_ports for s in specs])[ec]
    env = cx.Env(specs, env_class=ec, seed=seed)
    if not args.no_tune:
        env.autotune(32, os.path.join(ROOT, "gpurun_out", "autotune_cache.json")
                     if os.path.isdir(os.path.join(ROOT, "gpurun_out")) else None)
    out = env.alloc_traj(T, cx.OUT_FULL)
    stream = env.stream
    for _ in range(args.warmup):
        env.rollout(T, cx.ACT_RANDOM, cx.OUT_FULL, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        env.rollout(T, cx.ACT_RANDOM, cx.OUT_FULL, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    env_steps = N_ENVS * T
    value = env_steps / (ms_per_step / 1e3)
    alg_bytes = float((record_bytes(n_ports) * T + 2 * state_bytes(n_ports)).sum())
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9

    plain = None
    if not args.no_plain:
        out1 = env.alloc_traj(1, cx.OUT_FULL)
        for _ in range(8):
            env.step(cx.ACT_RANDOM, out=out1)
        torch.cuda.synchronize()
        reps = 2
        t1 = time.perf_counter()
        for _ in range(reps * T):
            env.step(cx.ACT_RANDOM, out=out1)
        torch.cuda.synchronize()
        p_ms = (time.perf_counter() - t1) * 1e3 / reps
        plain = {"ms_per_rollout": p_ms, "env_steps_per_s": env_steps / (p_ms / 1e3),
                 "launches_per_rollout": T}

    cpu = None if args.no_cpu else cpu_baseline(specs, ec, seed)
    ci = [env.class_info(c) for c in range(len(specs))]
    line = {
        "metric": "env-steps/s (batched persistent rollout, uneven stations)",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uneven-batching: 65536 stations x 288 steps, ports {8..128} mix, "
                               "trees depth 1-3, random levels, full records",
                   "n_envs": N_ENVS, "T": T, "mean_ports": float(n_ports.mean()),
                   "packing": {f"N{c.n_ports}d{c.levels}": c.lanes_per_station for c in ci},
                   "waves_per_block": ci[0].waves_per_block},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_rollout", "kernel_ms": kernel_ms, "algorithmic_bytes": alg_bytes},
        "plain": plain,
        "speedup_vs_plain": (value / plain["env_steps_per_s"]) if plain else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
