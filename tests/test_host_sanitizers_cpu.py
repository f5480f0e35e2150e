"""Host code under sanitizers, on the CPU.

The library's host code (contexts, tree compiler, tables, snapshots, the
autotuner's search and cache, the policy loop and the serving scheduler) is
built for the host only and linked against a fake HIP device (tests/sanitize):
device memory is host memory, a device thread runs the queued work in order
after random delays, and a kernel "runs" by checking every range its launch
arguments make it read or write.  The driver runs the whole C ABI on it, once
under AddressSanitizer + UndefinedBehaviorSanitizer (memory errors, leaks,
undefined behaviour) and once under ThreadSanitizer (the server's scheduler
thread against four client threads).  Two self-checks show that the fake
device refuses a launch into a buffer one step too short and into a freed
buffer.  The FP64 oracle runs a multi-threaded rollout under ASan + UBSan too.
"""
import os
import subprocess
import sys

import pytest

from tests.sanitize import build as SB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitize")
    scen = str(d / "scenario.txt")
    SB.write_scenario(scen)
    return {"asan": SB.build("asan", str(d / "asan")), "tsan": SB.build("tsan", str(d / "tsan")),
            "scenario": scen, "dir": d}


def run(cmd, env_extra, timeout=600):
    env = dict(os.environ, **env_extra)
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_asan_ubsan_whole_abi(drivers):
    cache = str(drivers["dir"] / "tune_asan.json")
    rc, out = run([drivers["asan"], drivers["scenario"], cache], {"ASAN_OPTIONS": "detect_leaks=1"})
    assert rc == 0 and "DRIVE OK" in out, out[-4000:]
    assert "graph execs destroyed with launches in flight: 0" in out
    assert "device allocations left: 0" in out
    assert os.path.getsize(cache) > 0          # the tuner searched and wrote its cache


def test_tsan_whole_abi(drivers):
    cache = str(drivers["dir"] / "tune_tsan.json")
    rc, out = run([drivers["tsan"], drivers["scenario"], cache], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert rc == 0 and "DRIVE OK" in out and "WARNING: ThreadSanitizer" not in out, out[-4000:]


@pytest.mark.parametrize("check", ["--undersized", "--freed"])
def test_fake_device_refuses_bad_launches(drivers, check):
    rc, out = run([drivers["asan"], drivers["scenario"], str(drivers["dir"] / "c.json"), check],
                  {"ASAN_OPTIONS": "detect_leaks=0"})
    assert rc != 0 and "FAKE-HIP ERROR" in out and "observations" in out, out[-2000:]


def test_oracle_asan_ubsan(tmp_path):
    so = str(tmp_path / "libcx_oracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-ffp-contract=off", "-fPIC", "-shared", "-pthread", "-o", so,
                           os.path.join(ROOT, "oracle", "cx_oracle.c"), "-lm"])
    script = f"""
import sys
import numpy as np
sys.path.insert(0, {ROOT!r})
from oracle import oracle as o
o._SO = {so!r}
import workloads as W
specs = W.mixture_classes() + [W.two_charger_types(), W.v2g_station(), W.exo_station(), W.user_station(),
                               W.fanout4_tree(256, 4, factor=0.6)]
counts = [5, 3, 7, 9, 1, 6, 4, 11, 2, 3, 5, 1, 2, 1, 3, 6, 5, 4, 3, 2]
ec = np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(counts)])
bs = o.BatchState([o.OracleClass(s) for s in specs], ec)
o.rollout(bs, 44, 300, want_info=True, n_threads=7)
o.rollout(bs, 44, 40, mode=2, n_threads=3)
c = o.OracleClass(W.policy_station())
c.policy(256, W.policy_weights(32, hidden=256, seed=3), c.observe(o.EnvState(32)), 5, 0, 0)
print("ORACLE OK")
"""
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    rc, out = run([sys.executable, "-c", script], {"LD_PRELOAD": libasan, "ASAN_OPTIONS": "detect_leaks=0"})
    assert rc == 0 and "ORACLE OK" in out, out[-4000:]
