"""GPU parity of charge-sensitive users (u = 1; the extended kernels) against the
FP64 oracle: user types, departures, c_satisfaction,1, observations and state.
The departure of such a user is decided by a float reaching zero; where the two
sides part because that decision fell within rounding of zero, the env is
accepted only if the oracle shows the near-tie (tests/parity.py), and such
flips must stay rare."""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu


def user_classes():
    return [W.scale_station().replace(charge_sensitive_share=0.5, alpha_sat1=0.3, beta_sat1=0.4, alpha_sat=0.1,
                                      arrival_peak=1.2, name="split16_cs50"),
            W.v2g_station().replace(charge_sensitive_share=0.3, alpha_sat1=0.2, beta_sat1=0.5,
                                    alpha_degrad_cars=0.02, name="v2g_batt_cs30"),
            W.two_charger_types().replace(charge_sensitive_share=1.0, alpha_sat1=0.1, beta_sat1=0.0,
                                          name="types_cs100"),
            W.fanout4_tree(40, 3).replace(charge_sensitive_share=0.7, alpha_sat1=0.05, beta_sat1=1.0,
                                          arrival_peak=2.0, name="fan40_cs70"),
            W.tiny_parity_station()]


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def ec_of(counts):
    return np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(counts)])


def run_checked(cxm, o, specs, ec, seed, T, mode, act_in=None, lanes=None, wpb=4):
    env = cxm.Env(specs, env_class=ec, seed=seed) if len(specs) > 1 else cxm.Env(specs[0], n_envs=len(ec), seed=seed)
    if lanes is not None:
        for c, L in enumerate(lanes):
            env.set_packing(c, L, wpb)
    bs = o.BatchState([o.OracleClass(s) for s in specs], ec)
    ain = None if act_in is None else torch.from_numpy(act_in).cuda()
    g = PY.to_np(env.rollout(T, mode, cxm.OUT_FULL, actions=ain))
    r = o.rollout(bs, seed, T, mode=mode, act_in=act_in)
    flips, keep = PY.compare_rollout_flips(o, g, r, specs, ec, seed, mode=mode, act_in=act_in)
    assert len(flips) <= max(1, len(ec) // 50), flips
    PY.compare_state(env.state_arrays(), bs, specs, ec, keep=keep)
    return env, g, flips


def test_mixed_launch_random(cxm, oracle_lib):
    """Four classes with charge-sensitive users (one with V2G and a battery, one
    with every user charge-sensitive) and a plain class in one launch, 300 steps."""
    specs = user_classes()
    ec = ec_of([41, 23, 17, 19, 9])
    env, g, flips = run_checked(cxm, oracle_lib, specs, ec, 31, 300, cxm.ACT_RANDOM)
    # overstaying users were seen: negative time left in the observations of class 0
    _, oo = PY.env_layout(specs, ec)
    N = specs[0].n_ports
    assert (g["obs"][:, oo[0] + 3 * N:oo[0] + 4 * N] < 0).any()
    assert g["obs"][:, oo[0] + 6 * N + 4:oo[0] + 7 * N + 4].max() == 1.0     # user flags


def test_low_and_max_levels(cxm, oracle_lib):
    """Level 1 everywhere (users overstay until charged) and the max-charge mode
    (users leave early)."""
    specs = user_classes()[:4]
    ec = ec_of([13, 9, 7, 11])
    T = 200
    n_act = sum(specs[c].n_actions for c in ec)
    low = np.full((T, n_act), 1, np.uint8)
    ao, _ = PY.env_layout(specs, ec)
    for e in np.flatnonzero(ec == 1):            # V2G class: byte 11 = level 1
        low[:, ao[e]:ao[e + 1]] = 11
    run_checked(cxm, oracle_lib, specs, ec, 32, T, cxm.ACT_EXTERNAL, act_in=low)
    run_checked(cxm, oracle_lib, specs, ec, 33, T, cxm.ACT_MAX)


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_packings(cxm, oracle_lib, lanes):
    specs = [user_classes()[0]]
    run_checked(cxm, oracle_lib, specs, np.zeros(37, np.int32), 34, 150, cxm.ACT_RANDOM, lanes=[lanes], wpb=2)


def test_plain_snapshot_observe(cxm):
    specs = user_classes()
    ec = ec_of([7, 5, 4, 6, 3])
    a = cxm.Env(specs, env_class=ec, seed=35)
    b = cxm.Env(specs, env_class=ec, seed=35)
    roll = PY.to_np(a.rollout(60, cxm.ACT_RANDOM))
    steps = [PY.to_np(b.step(cxm.ACT_RANDOM)) for _ in range(60)]
    for k in roll:
        assert np.array_equal(roll[k], np.concatenate([s[k] for s in steps])), k
    assert a.get_state() == b.get_state()
    assert torch.equal(a.observe(), torch.from_numpy(roll["obs"][-1]).cuda())
    snap = a.get_state()
    x = PY.to_np(a.rollout(80, cxm.ACT_RANDOM))
    a.set_state(snap)
    y = PY.to_np(a.rollout(80, cxm.ACT_RANDOM))
    for k in x:
        assert np.array_equal(x[k], y[k]), k
    st = a.state_arrays()
    assert (st["user"][st["dwell"] < 0] == 1).all()


def test_served_equals_direct(cxm):
    specs = user_classes()
    reqs = [(specs[0], 300, 320, 41), (specs[1], 90, 150, 42), (specs[4], 200, 100, 43)]
    srv = cxm.Server(2 << 30, chunk_steps=32)
    ts = [srv.submit(s, n, T, seed, cxm.OUT_FULL) for (s, n, T, seed) in reqs]
    for t, (s, n, T, seed) in zip(ts, reqs):
        got = srv.fetch(srv.wait(t), cxm.OUT_FULL, s)
        ref = PY.to_np(cxm.Env(s, n_envs=n, seed=seed).rollout(T, cxm.ACT_RANDOM, cxm.OUT_FULL))
        for k in got:
            assert np.array_equal(got[k], ref[k]), (t, k)
        srv.release(t)
    srv.close()


def test_full_size_sampled(cxm, oracle_lib):
    """65,536 stations (16 ports, half the users charge-sensitive) x 288 steps;
    48 sampled stations replayed in the oracle."""
    o = oracle_lib
    spec = W.user_station()
    n, T, seed = 65536, 288, 4
    env = cxm.Env(spec, n_envs=n, seed=seed)
    out = env.rollout(T, cxm.ACT_RANDOM)
    rng = np.random.default_rng(11)
    ids = np.unique(np.concatenate([rng.choice(n, 46, replace=False), [0, n - 1]]))
    acols = (ids[:, None] * spec.n_actions + np.arange(spec.n_actions)).ravel()
    ocols = (ids[:, None] * spec.obs_dim + np.arange(spec.obs_dim)).ravel()
    g = {"actions": out["actions"][:, torch.from_numpy(acols).cuda()].cpu().numpy(),
         "reward": out["reward"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "done": out["done"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "obs": out["obs"][:, torch.from_numpy(ocols).cuda()].cpu().numpy()}
    ec = np.zeros(len(ids), np.int32)
    bs = o.BatchState([o.OracleClass(spec)], ec, env_ids=ids)
    ref = o.rollout(bs, seed, T)
    first = PY.env_mismatch_steps(g, ref, [spec], ec)
    for e in np.flatnonzero(first < T):
        ties = PY.near_tie_steps(o, spec, seed, int(ids[e]), int(first[e]) + 1)
        assert any(first[e] - 2 <= s <= first[e] for s in ties), (ids[e], first[e])
    assert (first < T).sum() <= 1
