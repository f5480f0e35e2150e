"""Serving on the GPU: every request's records equal a direct rollout of the same
stations (same seed, same horizon) bit for bit, alone or mixed with requests of
other classes, sizes and horizons; and equal the oracle within the parity
tolerances."""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def direct(cxm, spec, n_envs, T, seed, out_mode, act_mode):
    env = cxm.Env(spec, n_envs=n_envs, seed=seed)
    out = PY.to_np(env.rollout(T, act_mode, out_mode))
    return out


def mixed_requests(cxm):
    A, M = cxm.ACT_RANDOM, cxm.ACT_MAX
    return [
        (W.scale_station(), 4096, 1500, 10, cxm.OUT_REWARD, A),   # long: the others join it
        (W.tiny_parity_station(), 64, 100, 11, cxm.OUT_FULL, A),
        (W.scale_station(), 200, 77, 12, cxm.OUT_ACT_REWARD, A),
        (W.fanout4_tree(32, 2), 33, 300, 13, cxm.OUT_REWARD, A),
        (W.tiny_parity_station(), 5, 40, 14, cxm.OUT_FULL, M),
        (W.fanout4_tree(128, 3), 17, 65, 15, cxm.OUT_FULL, A),
        (W.two_charger_types(), 50, 290, 16, cxm.OUT_FULL, A),
    ]


def test_served_equals_direct(cxm):
    """Seven requests of differing class, size, horizon, output and action mode
    run together (chunks of 32 steps): each equals its own direct rollout."""
    reqs = mixed_requests(cxm)
    srv = cxm.Server(8 << 30, chunk_steps=32)
    tickets = [srv.submit(s, n, T, seed, om, act_mode=am) for (s, n, T, seed, om, am) in reqs]
    for t, (s, n, T, seed, om, am) in zip(tickets, reqs):
        r = srv.wait(t)
        assert r.status == 0
        got = srv.fetch(r, om, s.n_ports)
        ref = direct(cxm, s, n, T, seed, om, am)
        for k in got:
            assert np.array_equal(got[k], ref[k]), (t, k)
        srv.release(t)
    st = srv.stats()
    assert st["env_steps"] == sum(n * T for (_, n, T, _, _, _) in reqs)
    assert st["peak_active"] >= 3          # the short requests ran alongside the long one
    srv.close()


def test_alone_equals_mixed_and_caller_buffers(cxm):
    """A request served alone with caller-owned output tensors equals the same
    request served in a mix with server-owned buffers; chunk size 7 (ragged)."""
    spec, n, T, seed = W.scale_station(), 96, 100, 21
    srv = cxm.Server(4 << 30, chunk_steps=7)
    out = {"obs": torch.empty((T, n * spec.obs_dim), dtype=torch.float32, device="cuda"),
           "actions": torch.empty((T, n * spec.n_ports), dtype=torch.uint8, device="cuda"),
           "reward": torch.empty((T, n), dtype=torch.float32, device="cuda"),
           "done": torch.empty((T, n), dtype=torch.uint8, device="cuda")}
    t = srv.submit(spec, n, T, seed, cxm.OUT_FULL, out=out)
    r = srv.wait(t)
    assert r.status == 0 and r.traj.obs == out["obs"].data_ptr()
    alone = PY.to_np(out)
    srv.release(t)
    others = [srv.submit(s, nn, TT, sd, om, act_mode=am) for (s, nn, TT, sd, om, am) in mixed_requests(cxm)[:4]]
    t2 = srv.submit(spec, n, T, seed, cxm.OUT_FULL)
    r2 = srv.wait(t2)
    mixed = srv.fetch(r2, cxm.OUT_FULL, spec.n_ports)
    for k in alone:
        assert np.array_equal(alone[k], mixed[k]), k
    for o in others:
        srv.wait(o)
        srv.release(o)
    srv.release(t2)
    srv.close()


def test_served_equals_oracle(cxm, oracle_lib):
    spec, n, T, seed = W.two_charger_types(), 40, 300, 31
    srv = cxm.Server(2 << 30, chunk_steps=64)
    t = srv.submit(spec, n, T, seed, cxm.OUT_FULL)
    got = srv.fetch(srv.wait(t), cxm.OUT_FULL, spec.n_ports)
    srv.release(t)
    srv.close()
    bs = oracle_lib.BatchState([oracle_lib.OracleClass(spec)], np.zeros(n, np.int32))
    ref = oracle_lib.rollout(bs, seed, T)
    PY.compare_rollout(got, ref, [spec], np.zeros(n, np.int32))


def test_cancel_running_on_gpu(cxm):
    spec = W.scale_station()
    srv = cxm.Server(8 << 30, chunk_steps=16)
    t = srv.submit(spec, 4096, 4000, 1, cxm.OUT_REWARD)
    srv.cancel(t)
    r = srv.wait(t)
    assert r.status in (-6, 0)
    srv.release(t)
    t2 = srv.submit(spec, 8, 20, 2, cxm.OUT_REWARD)
    assert srv.wait(t2).status == 0
    srv.release(t2)
    srv.close()
