"""Benchmark of batched EV charging-station rollouts on one MI355X.

Default workload (uneven batching): 65,536 stations whose port counts are drawn
from {8, 16, 32, 64, 128} with probabilities {.3, .3, .2, .15, .05}, capacity
trees 1-3 levels deep (fan-out 4, limits 0.7x the children's maxima), 288
five-minute steps, Philox random levels, every per-step record written
(observations, levels, rewards, done flags).  One bench "step" = one rollout of
all stations over all 288 steps in one persistent, graph-replayed launch.

Other workloads (--workload): tiny (64 stations of 16 ports, the parity case),
scale (4,096 stations on a two-level tree, persistent vs one launch per step),
v2g (65,536 stations with bidirectional ports and a station battery), users
(65,536 stations where half the users are charge-sensitive), exo (65,536
two-charger-type stations driven by an arrival table and 28 price days),
policy (1,048,576 stations of 32 ports, levels from the BF16 perceptron on the
matrix cores, the perceptron and the step fused in one persistent launch), serve (a Poisson stream of rollout requests through the
continuous-batching server).

Prints one JSON line: the throughput, the roofline of the dominant kernel, and
the FP64 oracle on the host's cores as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
T_DAY = 288
# steps per serving launch: on the serving stream, 144 beat 16, 32, 64, 96 and
# 288 in saturated throughput and in p99 latency (p50 within 2 % of the best)
SERVE_CHUNK = 144


def record_bytes(spec, out_mode: str = "full") -> int:
    """Bytes of one record per env-step: obs (obs_dim f32: 6N+4, +2 with a
    station battery, +2 with price days, +N with charge-sensitive users), one
    action byte per port (+1 for the battery), reward f32, done u8."""
    if out_mode == "full":
        return 4 * spec.obs_dim + spec.n_actions + 4 + 1
    if out_mode == "act_reward":
        return spec.n_actions + 4 + 1
    return 4 + 1


def state_bytes(spec) -> int:
    """Per env: 1 - SoC (f64), 1 - target, capacity, last power (f32) and dwell (i16)
    per port and the f64 return; with a battery its f64 SoC and f32 power, with
    charge-sensitive users a user byte per port, with car models the car's f32
    rate per port."""
    N = spec.n_ports
    return (22 * N + 8 + (12 if getattr(spec, "has_battery", False) else 0)
            + (N if getattr(spec, "has_users", False) else 0)
            + (4 * N if getattr(spec, "car_models", None) is not None else 0))


def rollout_bytes(specs, ec, T: int, out_mode: str = "full") -> float:
    """Algorithmic bytes of one T-step rollout: every record once, the state read
    once and written once."""
    counts = np.bincount(np.asarray(ec), minlength=len(specs))
    return float(sum(int(n) * (T * record_bytes(s, out_mode) + 2 * state_bytes(s)) for s, n in zip(specs, counts)))


def measured_traffic():
    """HBM bytes of one default rollout from the committed counter profile, if it
    was taken on the current kernel source (None otherwise)."""
    import hashlib
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "k_rollout_traffic.json")))
        src = open(os.path.join(ROOT, "paper_2507_01522_amd", "csrc", "cx_kernels.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest()[:16] != prof.get("kernel_sha256_prefix"):
        return None
    return float(prof["traffic_bytes"])


def uneven_workload():
    import workloads as W
    classes = W.mixture_classes()
    ec_full = W.mixture_env_classes(65536, seed=1003)
    return W.compact_classes(classes, ec_full)


def oracle_baseline(specs, ec, seed, T, stride, chunk=16, mode=1, min_s=10.0, threads=None):
    """The FP64 oracle on an evenly spaced sample of the same stations, whole days
    repeated until about min_s seconds of host time have passed; threads: host
    threads (default: the cores, at most 16)."""
    from oracle import oracle as o
    ids = np.arange(0, len(ec), stride, dtype=np.int64)
    classes = [o.OracleClass(s) for s in specs]
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    used, steps, days = 1, 0, 0
    out = None      # the output arrays are reused from chunk to chunk (no page faults in the timing)
    t0 = time.perf_counter()
    while True:
        bs = o.BatchState(classes, np.asarray(ec)[ids], env_ids=ids)
        for _ in range(max(1, T // chunk)):
            out = o.rollout(bs, seed, min(chunk, T), mode=mode, n_threads=threads, out=out)
            used = out["threads"]
            steps += min(chunk, T)
        days += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = time.perf_counter() - t0
    return {"value": len(ids) * steps / dt, "unit": "env-steps/s", "cores": int(used), "kind": "oracle",
            "sample": f"{len(ids)} of {len(ec)} stations (every {stride}th), {days} x {T} steps, FP64, "
                      f"all outputs, {used} threads, {dt:.1f} s"}


def time_events(fn, reps, stream):
    """Mean milliseconds of fn() between HIP events on ``stream`` (after one warm-up)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def base_line(metric, value, unit, args, ms_per_step, config, dtype="f32"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def timed_rollouts(env, cx, T, mode, out_mode, out, args):
    """W untimed + K timed rollouts; returns (wall ms per rollout, event ms per rollout)."""
    import torch
    stream = env.stream
    for _ in range(args.warmup):
        env.rollout(T, mode, out_mode, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        env.rollout(T, mode, out_mode, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def plain_rate(env, cx, n_envs, T, reps=2):
    """The same rollout as T one-step launches (state through HBM every step)."""
    import torch
    out1 = env.alloc_traj(1, cx.OUT_FULL)
    for _ in range(8):
        env.step(cx.ACT_RANDOM, out=out1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps * T):
        env.step(cx.ACT_RANDOM, out=out1)
    torch.cuda.synchronize()
    p_ms = (time.perf_counter() - t1) * 1e3 / reps
    return {"ms_per_rollout": p_ms, "env_steps_per_s": n_envs * T / (p_ms / 1e3), "launches_per_rollout": T}


def run_rollout_workload(args, name, specs, ec, seed, desc, cpu_stride):
    import torch  # noqa: F401
    import paper_2507_01522_amd as cx
    n_ports = np.array([s.n_ports for s in specs])[ec]
    n_envs = len(ec)
    from paper_2507_01522_amd.launch import configure
    env = cx.Env(specs, env_class=ec, seed=seed) if len(specs) > 1 else cx.Env(specs[0], n_envs=n_envs, seed=seed)
    configure(env, name, len(specs))
    out = env.alloc_traj(T_DAY, cx.OUT_FULL)
    wall_ms, kernel_ms = timed_rollouts(env, cx, T_DAY, cx.ACT_RANDOM, cx.OUT_FULL, out, args)
    env_steps = n_envs * T_DAY
    value = env_steps / (wall_ms / 1e3)
    alg_bytes = rollout_bytes(specs, ec, T_DAY, "full")
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    del out
    # records of rewards and done flags only (the same rollout, 5 bytes per env-step)
    out_r = env.alloc_traj(T_DAY, cx.OUT_REWARD)
    r_wall, r_kernel = timed_rollouts(env, cx, T_DAY, cx.ACT_RANDOM, cx.OUT_REWARD, out_r, args)
    del out_r
    plain = None if args.no_plain else plain_rate(env, cx, n_envs, T_DAY)
    cpu = None if args.no_cpu else oracle_baseline(specs, ec, seed, T_DAY, cpu_stride)
    ci = [env.class_info(c) for c in range(len(specs))]
    line = base_line(f"env-steps/s (batched persistent rollout, {desc})", value, "env-steps/s", args, wall_ms,
                     {"workload": name, "n_envs": n_envs, "T": T_DAY, "mean_ports": float(n_ports.mean()),
                      "packing": {f"N{c.n_ports}d{c.levels}": c.lanes_per_station for c in ci},
                      "waves_per_block": ci[0].waves_per_block,
                      "obs_stage": bool(env.info().obs_stage)})
    line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic() if name.startswith("uneven") else None,
                        "kernel": "k_rollout", "kernel_ms": kernel_ms, "algorithmic_bytes": alg_bytes}
    line["reward_only"] = {"env_steps_per_s": env_steps / (r_wall / 1e3), "kernel_ms": r_kernel,
                           "algorithmic_bytes": rollout_bytes(specs, ec, T_DAY, "reward")}
    line["plain"] = plain
    line["speedup_vs_plain"] = (value / plain["env_steps_per_s"]) if plain else None
    line["cpu_baseline"] = cpu
    return line


def run_uneven(args):
    specs, ec = uneven_workload()
    line = run_rollout_workload(
        args, "uneven-batching: 65536 stations x 288 steps, ports {8..128} mix, trees depth 1-3, random "
              "levels, full records", specs, ec, 3, "uneven stations", 8)
    if not args.no_serve:
        line["serve"] = serve_fixed_rate()
    return line


def run_tiny(args):
    import workloads as W
    return run_rollout_workload(args, "tiny: 64 stations x 288 steps, 16 ports under 150 kW, random levels, "
                                      "full records", [W.tiny_parity_station()], np.zeros(64, np.int32), 1,
                                "64 stations", 1)


def run_scale(args):
    import workloads as W
    return run_rollout_workload(args, "scale: 4096 stations x 288 steps, 4 splitters x 4 ports of 22 kW, "
                                      "random levels, full records", [W.scale_station()],
                                np.zeros(4096, np.int32), 2, "4096 stations", 4)


def run_v2g(args):
    import workloads as W
    return run_rollout_workload(args, "v2g: 65536 stations x 288 steps, 4 splitters x 4 bidirectional 22 kW "
                                      "ports, 200 kWh / 50 kW station battery, random signed levels, full "
                                      "records", [W.v2g_station()], np.zeros(65536, np.int32), 3,
                                "V2G stations with batteries", 64)


def run_users(args):
    import workloads as W
    return run_rollout_workload(args, "users: 65536 stations x 288 steps, 4 splitters x 4 ports of 22 kW, half "
                                      "the users charge-sensitive (leave when charged), random levels, full "
                                      "records", [W.user_station()], np.zeros(65536, np.int32), 4,
                                "stations with charge-sensitive users", 64)


def run_exo(args):
    import workloads as W
    return run_rollout_workload(args, "exo: 65536 stations x 288 steps, 10 DC + 6 AC ports under per-type splitters, "
                                      "commuter arrival table, exploring starts over 28 price days, European car "
                                      "mix (AC / DC rates), random levels, full records", [W.exo_station()], np.zeros(65536, np.int32), 5,
                                "table-driven stations", 64)


def run_policy(args):
    """Policy in the loop: one launch of the fused rollout kernel runs, every
    step, the environment step and the perceptron that samples every port's
    level for the next step (the observation kernel gives the first step's
    input)."""
    import torch
    import paper_2507_01522_amd as cx
    import workloads as W
    spec = W.policy_station()
    E, H, seed = 1 << 20, 256, 5
    N, dim = spec.n_ports, spec.obs_dim
    weights = W.policy_weights(N, hidden=H)
    env = cx.Env(spec, n_envs=E, seed=seed)
    env.set_policy(H, weights)
    out = env.alloc_traj(T_DAY, cx.OUT_ACT_REWARD)
    wall_ms, ev_ms = timed_rollouts(env, cx, T_DAY, cx.ACT_POLICY, cx.OUT_ACT_REWARD, out, args)
    value = E * T_DAY / (wall_ms / 1e3)
    # algorithmic matrix-core work of the rollout: both products, every env-step
    flops = 2.0 * E * T_DAY * (dim * H + H * N * (spec.n_levels + 1))
    achieved = flops / (ev_ms / 1e3) / 1e12
    # the standalone policy kernel (one step of observations in, levels out),
    # timed alone for comparison: the two-kernel path of other classes
    obs = env.observe().view(E, dim)
    act = torch.empty((E, N), dtype=torch.uint8, device=env.device)
    pol_ms = time_events(lambda: env.policy_sample(obs, 7, act), 10, env.stream)
    cpu = None
    if not args.no_cpu:
        cpu = policy_oracle_baseline(spec, H, weights, seed)
    line = base_line("env-steps/s (policy-in-the-loop rollout)", value, "env-steps/s", args, wall_ms,
                     {"workload": "policy: 1048576 stations x 288 steps, 32 ports (8 splitters x 4 under "
                                  "400 kW), MLP 196-256-352 BF16, levels drawn from softmax, levels+rewards",
                      "n_envs": E, "T": T_DAY, "hidden": H, "kernel": "fused (8 lanes x 4 slots, 4 waves per block)"},
                     dtype="bf16")
    line["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None, "kernel": "k_rollout_policy<8, 4>",
                        "kernel_ms": ev_ms, "algorithmic_flops": flops,
                        "note": "HIP-event time of the rollout: the fused kernel plus the observation kernel of "
                                "the start state (well under 1 %)"}
    step_flops = flops / T_DAY
    line["standalone_policy_kernel"] = {"kernel": "k_policy", "ms_per_step": pol_ms,
                                        "achieved_TFLOPs": step_flops / (pol_ms / 1e3) / 1e12}
    line["cpu_baseline"] = cpu
    return line


def policy_oracle_baseline(spec, H, weights, seed, n_envs=64, min_s=10.0):
    """The oracle's policy and transition, one env-step at a time, on 64 stations,
    steps repeated until about min_s seconds of host time have passed."""
    from oracle import oracle as o
    c = o.OracleClass(spec)
    N = spec.n_ports
    bs = o.BatchState([c], np.zeros(n_envs, np.int32))
    t0 = time.perf_counter()
    st = o.EnvState(N)
    obs = np.stack([c.observe(st)] * n_envs)
    t = 0
    while True:
        act = np.stack([c.policy(H, weights, obs[e], seed, e, t)[1] for e in range(n_envs)]).astype(np.uint8)
        out = o.rollout(bs, seed, 1, mode=0, act_in=act.reshape(1, -1), n_threads=1)
        obs = out["obs"].reshape(n_envs, -1)
        t += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n_envs * t / dt, "unit": "env-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_envs} stations x {t} steps of the policy workload, FP64 perceptron + step, "
                      f"1 thread, {dt:.1f} s"}


def serve_requests(srv, classes, reqs, paced):
    """Submit requests (paced by their arrival times, or all at once); a client
    thread polls the outstanding tickets and releases each as soon as it
    finishes.  Returns (wall s, server stats of this run, latencies s, queueing s)."""
    import paper_2507_01522_amd as cx
    st0 = srv.stats()
    lat, admit_wait = [], []
    lock = threading.Lock()
    outstanding = []

    def drain():
        n_done = 0
        while n_done < len(reqs):
            with lock:
                live = list(outstanding)
            finished = []
            for tk in live:
                r = srv.poll(tk)
                if r is None:
                    continue
                lat.append(r.done_s - r.submit_s)
                admit_wait.append(r.admit_s - r.submit_s)
                srv.release(tk)
                finished.append(tk)
            if finished:
                with lock:
                    for tk in finished:
                        outstanding.remove(tk)
                n_done += len(finished)
            else:
                time.sleep(0.0005)

    th = threading.Thread(target=drain)
    th.start()
    t0 = time.perf_counter()
    for rq in reqs:
        if paced:
            d = rq.arrival_s - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
        tk = srv.submit(classes[rq.class_index], rq.n_envs, rq.horizon, rq.seed, cx.OUT_FULL)
        with lock:
            outstanding.append(tk)
    th.join()
    wall = time.perf_counter() - t0
    st1 = srv.stats()
    st = {k: st1[k] - st0[k] for k in ("busy_s", "env_steps", "launches")}
    st["peak_active"] = st1["peak_active"]
    return wall, st, np.array(lat), np.array(admit_wait)


def serve_summary(classes, stream, wall, st, lat, wq, rate):
    env_steps = sum(r.n_envs * r.horizon for r in stream)
    rec = {c: record_bytes(classes[c]) for c in range(len(classes))}
    alg = float(sum(r.n_envs * (r.horizon * rec[r.class_index] + 2 * state_bytes(classes[r.class_index]))
                    for r in stream))
    return {"rate_req_per_s": rate, "requests": len(stream), "env_steps_per_s": env_steps / wall,
            "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "queue_p50": float(np.percentile(wq, 50)), "queue_p99": float(np.percentile(wq, 99))},
            "gpu_busy_s": st["busy_s"], "hbm_GBps_of_busy_time": alg / st["busy_s"] / 1e9,
            "peak_active": st["peak_active"], "algorithmic_bytes": alg, "wall_s": wall}


def serve_fixed_rate(rate=1000.0, n=400, seed=2003):
    """The serving loop at a fixed Poisson request rate (continuous batching,
    chunks of SERVE_CHUNK steps, 200 GB budget): p50/p99 latency and
    env-steps/s, for the default bench line."""
    import paper_2507_01522_amd as cx
    import workloads as W
    classes = W.mixture_classes()
    srv = cx.Server(200 << 30, chunk_steps=SERVE_CHUNK)
    serve_requests(srv, classes, W.request_stream(40, 1e9, seed=2002), False)   # warm-up
    stream = W.request_stream(n, rate, seed=seed)
    wall, st, lat, wq = serve_requests(srv, classes, stream, True)
    srv.close()
    out = serve_summary(classes, stream, wall, st, lat, wq, rate)
    out["workload"] = (f"{n} Poisson requests at {rate:g}/s, 64..8192 stations, T in {{96,288,2016}}, "
                       "uneven classes, full records, 200 GB budget")
    return out


def run_serve(args):
    """A Poisson stream of rollout requests (log-uniform sizes 64..8192 stations,
    horizons {96, 288, 2016}, classes of the uneven mixture, full records) at
    0.7x the measured saturated request rate, 200 GB budget."""
    import paper_2507_01522_amd as cx
    import workloads as W
    classes = W.mixture_classes()
    srv = cx.Server(200 << 30, chunk_steps=SERVE_CHUNK)   # reserves the budget on the device once
    # saturated: bursts of requests submitted at once (the better of two)
    burst = W.request_stream(600, 1e9, seed=2001)
    serve_requests(srv, classes, W.request_stream(40, 1e9, seed=2002), False)   # warm-up
    wall_s = min(serve_requests(srv, classes, burst, False)[0] for _ in range(2))
    steps_s = sum(r.n_envs * r.horizon for r in burst)
    sat_rate = len(burst) / wall_s
    rate = 0.7 * sat_rate
    stream = W.request_stream(1000, rate, seed=2000)
    wall, st, lat, wq = serve_requests(srv, classes, stream, True)
    srv.close()
    sm = serve_summary(classes, stream, wall, st, lat, wq, rate)
    line = base_line("env-steps/s (continuous-batching server, Poisson request stream)", sm["env_steps_per_s"],
                     "env-steps/s", args, wall * 1e3,
                     {"workload": "serve: 1000 Poisson requests at 0.7x saturated rate, 64..8192 stations, "
                                  "T in {96,288,2016}, uneven classes, full records, 200 GB budget",
                      "rate_req_per_s": rate, "saturated_req_per_s": sat_rate,
                      "saturated_env_steps_per_s": steps_s / wall_s, "chunk_steps": SERVE_CHUNK})
    line["latency_s"] = sm["latency_s"]
    line["server"] = st
    line["roofline"] = {"bound": "hbm", "achieved": sm["hbm_GBps_of_busy_time"], "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": sm["hbm_GBps_of_busy_time"] / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "k_rollout (per-segment chunks)", "kernel_ms": st["busy_s"] * 1e3,
                        "algorithmic_bytes": sm["algorithmic_bytes"]}
    line["cpu_baseline"] = None
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uneven", choices=["uneven", "tiny", "scale", "v2g", "users", "exo", "policy", "serve"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-step comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement of the default line")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 2 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the rollout has no cross-GPU work; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calib_copy:
        src = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    run = {"uneven": run_uneven, "tiny": run_tiny, "scale": run_scale, "v2g": run_v2g, "users": run_users, "exo": run_exo,
           "policy": run_policy,
           "serve": run_serve}[args.workload]
    print(json.dumps(run(args)))


if __name__ == "__main__":
    main()
