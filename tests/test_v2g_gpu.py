"""GPU parity of V2G discharge and the station battery (the bidirectional
kernels) against the FP64 oracle: integers (action bytes, done flags, dwell)
bit-exact, FP values within the tolerances of tests/parity.py.  Bidirectional
classes share a launch with charging-only ones, run in every packing, in the
plain one-step form, through snapshots, resets, the observation kernel and the
server."""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu

V2G = W.v2g_mixture()
MIXED = V2G + [W.tiny_parity_station()]       # plus a charging-only class in the same launch
COUNTS = [37, 21, 13, 9, 26, 11]


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def make_env(cxm, specs, ec, seed):
    ec = np.asarray(ec, np.int32)
    if len(specs) == 1:
        return cxm.Env(specs[0], n_envs=len(ec), seed=seed)
    return cxm.Env(specs, env_class=ec, seed=seed)


def run_both(cxm, o, specs, ec, seed, T, mode, act_in=None, lanes=None, wpb=4):
    ec = np.asarray(ec, np.int32)
    env = make_env(cxm, specs, ec, seed)
    if lanes is not None:
        for c, L in enumerate(lanes):
            env.set_packing(c, L, wpb)
    bs = o.BatchState([o.OracleClass(s) for s in specs], ec)
    ain = None if act_in is None else torch.from_numpy(act_in).cuda()
    g = PY.to_np(env.rollout(T, mode, cxm.OUT_FULL, actions=ain))
    r = o.rollout(bs, seed, T, mode=mode, act_in=act_in)
    return env, bs, g, r


def ec_of(counts):
    return np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(counts)])


def test_mixed_launch_random(cxm, oracle_lib):
    """Five bidirectional classes and a charging-only one, ragged env counts,
    300 steps across the day boundary, random signed levels, every output."""
    ec = ec_of(COUNTS)
    env, bs, g, r = run_both(cxm, oracle_lib, MIXED, ec, 11, 300, cxm.ACT_RANDOM)
    PY.compare_rollout(g, r, MIXED, ec)
    PY.compare_state(env.state_arrays(), bs, MIXED, ec)
    info = env.info()
    assert info.total_ports == sum(MIXED[c].n_actions for c in ec)
    assert info.obs_elems == sum(MIXED[c].obs_dim for c in ec)
    assert g["done"][287].all() and g["done"].sum() == len(ec)
    # discharging happened: negative last powers in the observations of V2G ports
    _, oo = PY.env_layout(MIXED, ec)
    e = int(np.flatnonzero(ec == 0)[0])
    N = MIXED[0].n_ports
    assert (g["obs"][:, oo[e] + 5 * N:oo[e] + 6 * N] < 0).any()


def test_external_bytes_and_max(cxm, oracle_lib):
    """Caller action bytes (above the top byte: clamped) and the max-charge mode."""
    ec = ec_of([9, 5, 7, 3, 6, 4])
    T = 120
    n_act = sum(MIXED[c].n_actions for c in ec)
    act = np.random.default_rng(3).integers(0, 26, size=(T, n_act), dtype=np.uint8)
    env, bs, g, r = run_both(cxm, oracle_lib, MIXED, ec, 12, T, cxm.ACT_EXTERNAL, act_in=act)
    PY.compare_rollout(g, r, MIXED, ec)
    PY.compare_state(env.state_arrays(), bs, MIXED, ec)
    env, bs, g, r = run_both(cxm, oracle_lib, MIXED, ec, 13, 150, cxm.ACT_MAX)
    PY.compare_rollout(g, r, MIXED, ec)
    PY.compare_state(env.state_arrays(), bs, MIXED, ec)


@pytest.mark.parametrize("ports", [16, 64, 128])
def test_every_packing(cxm, oracle_lib, ports):
    """Bidirectional trees (with a battery) in every legal packing, 1 and 4 waves per block."""
    specs = [W.fanout4_tree(ports, d).replace(v2g=1, battery_kwh=100.0, battery_kw=40.0, battery_soc0=0.6,
                                               alpha_degrad_cars=0.02, alpha_degrad_battery=0.01)
             for d in (1, 2, 3)]
    ec = np.repeat(np.arange(3, dtype=np.int32), [11, 6, 8])
    for L in (4, 8, 16, 32, 64):
        if ports % L or ports // L not in (1, 2, 4):
            continue
        for wpb in (1, 4):
            env, bs, g, r = run_both(cxm, oracle_lib, specs, ec, 14, 100, cxm.ACT_RANDOM,
                                     lanes=[L] * 3, wpb=wpb)
            PY.compare_rollout(g, r, specs, ec)
            PY.compare_state(env.state_arrays(), bs, specs, ec)


def test_plain_steps_equal_persistent(cxm):
    ec = ec_of([5, 4, 3, 2, 6, 3])
    a = make_env(cxm, MIXED, ec, 15)
    b = make_env(cxm, MIXED, ec, 15)
    T = 40
    roll = PY.to_np(a.rollout(T, cxm.ACT_RANDOM))
    steps = [PY.to_np(b.step(cxm.ACT_RANDOM)) for _ in range(T)]
    for k in roll:
        assert np.array_equal(roll[k], np.concatenate([s[k] for s in steps])), k
    assert a.get_state() == b.get_state()


def test_snapshot_reset_observe(cxm, oracle_lib):
    """Snapshots carry the batteries; reset returns them to their initial SoC;
    the observation kernel equals the last record bit for bit."""
    o = oracle_lib
    ec = ec_of([8, 4, 6, 3, 5, 4])
    env = make_env(cxm, MIXED, ec, 16)
    env.rollout(70, cxm.ACT_RANDOM)
    snap = env.get_state()
    a = PY.to_np(env.rollout(60, cxm.ACT_RANDOM))
    assert torch.equal(env.observe(), torch.from_numpy(a["obs"][-1]).cuda())
    env.set_state(snap)
    b = PY.to_np(env.rollout(60, cxm.ACT_RANDOM))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    obs = torch.full((env.info().obs_elems,), 3.0, device="cuda")
    env.reset(obs)
    st = env.state_arrays()
    soc0 = np.array([MIXED[c].battery_soc0 if MIXED[c].has_battery else 0.0 for c in ec])
    assert np.array_equal(st["batt_soc"], soc0) and (st["batt_p"] == 0).all()
    ref = np.concatenate([o.OracleClass(MIXED[c]).observe(o.OracleClass(MIXED[c]).new_state()) for c in ec])
    PY.compare_obs(obs.cpu().numpy()[None], ref[None], MIXED, ec)
    assert torch.equal(env.observe(), obs)


def test_served_equals_direct_and_oracle(cxm, oracle_lib):
    """Bidirectional requests served alongside charging-only ones equal their
    direct rollouts bit for bit, and the oracle within tolerance."""
    reqs = [(V2G[0], 300, 400, 21), (W.scale_station(), 500, 300, 22), (V2G[2], 70, 150, 23),
            (V2G[4], 33, 97, 24)]
    srv = cxm.Server(4 << 30, chunk_steps=32)
    tickets = [srv.submit(s, n, T, seed, cxm.OUT_FULL) for (s, n, T, seed) in reqs]
    for t, (s, n, T, seed) in zip(tickets, reqs):
        r = srv.wait(t)
        assert r.status == 0
        got = srv.fetch(r, cxm.OUT_FULL, s)
        ref = PY.to_np(cxm.Env(s, n_envs=n, seed=seed).rollout(T, cxm.ACT_RANDOM, cxm.OUT_FULL))
        for k in got:
            assert np.array_equal(got[k], ref[k]), (t, k)
        srv.release(t)
        if s.v2g or s.has_battery:
            ec = np.zeros(n, np.int32)
            bs = oracle_lib.BatchState([oracle_lib.OracleClass(s)], ec)
            PY.compare_rollout(got, oracle_lib.rollout(bs, seed, T), [s], ec)
    srv.close()


def test_full_size_sampled(cxm, oracle_lib):
    """65,536 V2G stations with batteries x 288 steps in the default packing (16
    lanes, 4 waves per block; the measured launch is covered by
    test_fullsize_gpu): every action byte's range and done flag, and 48 sampled
    stations replayed in the oracle (actions, rewards, observations)."""
    o = oracle_lib
    spec = W.v2g_station()
    n, T, seed = 65536, 288, 3
    env = cxm.Env(spec, n_envs=n, seed=seed)
    out = env.rollout(T, cxm.ACT_RANDOM)
    a = out["actions"]
    assert int(a.max()) == 20 and int(a.min()) == 0
    assert bool(out["done"][-1].all()) and not bool(out["done"][:-1].any())
    rng = np.random.default_rng(9)
    ids = np.unique(np.concatenate([rng.choice(n, 46, replace=False), [0, n - 1]]))
    acols = (ids[:, None] * spec.n_actions + np.arange(spec.n_actions)).ravel()
    ocols = (ids[:, None] * spec.obs_dim + np.arange(spec.obs_dim)).ravel()
    g = {"actions": a[:, torch.from_numpy(acols).cuda()].cpu().numpy(),
         "reward": out["reward"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "done": out["done"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "obs": out["obs"][:, torch.from_numpy(ocols).cuda()].cpu().numpy()}
    ec = np.zeros(len(ids), np.int32)
    bs = o.BatchState([o.OracleClass(spec)], ec, env_ids=ids)
    PY.compare_rollout(g, o.rollout(bs, seed, T), [spec], ec)


def test_policy_rejects_bidirectional(cxm):
    spec = W.v2g_station()
    env = cxm.Env(spec, n_envs=4, seed=1)
    with pytest.raises(cxm.CxError):
        env.set_policy(256, W.policy_weights(spec.n_ports, hidden=256, seed=1))
