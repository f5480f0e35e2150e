"""The benchmark's host side: algorithmic bytes per rollout (records once, state
read and written once) for every workload, and the one-GPU contract."""
import subprocess
import sys
import os

import numpy as np

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_record_and_state_bytes():
    s = W.tiny_parity_station()                        # 16 ports: obs 100 f32, 16 levels, reward, done
    assert bench.record_bytes(s) == 4 * 100 + 16 + 5
    assert bench.record_bytes(s, "act_reward") == 16 + 5 and bench.record_bytes(s, "reward") == 5
    assert bench.state_bytes(s) == 22 * 16 + 8
    v = W.v2g_station()                                # + battery: 2 obs floats, 1 action byte, 12 state bytes
    assert bench.record_bytes(v) == 4 * 102 + 17 + 5 and bench.state_bytes(v) == 22 * 16 + 8 + 12
    u = W.user_station()                               # + 16 user flags and 16 user bytes
    assert bench.record_bytes(u) == 4 * 116 + 16 + 5 and bench.state_bytes(u) == 22 * 16 + 8 + 16
    e = W.exo_station()                                # + day features; + car rates in the state
    assert bench.record_bytes(e) == 4 * 102 + 16 + 5 and bench.state_bytes(e) == 22 * 16 + 8 + 64


def test_workload_bytes():
    specs, ec = bench.uneven_workload()
    assert bench.rollout_bytes(specs, ec, 288) == 14565341408.0
    assert bench.rollout_bytes(specs, ec, 288, "reward") == 181476320.0
    z = np.zeros(65536, np.int64)
    assert bench.rollout_bytes([W.v2g_station()], z, 288) == 8164737024.0
    assert bench.rollout_bytes([W.user_station()], z, 288) == 9203351552.0
    assert bench.rollout_bytes([W.exo_station()], z, 288) == 8152678400.0
    assert bench.rollout_bytes([W.policy_station()], np.zeros(1 << 20, np.int64), 1) == 2354053120.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
