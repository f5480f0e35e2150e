"""GPU parity of exploring starts (per-episode price days, Supp. B.1) and of the
table-driven exogenous station (commuter arrivals + price days), alone and
with V2G, a battery and charge-sensitive users, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu


def day_classes():
    days = W.price_day_table(9, seed=5)
    return [W.exo_station(alpha_sat=0.1),
            W.v2g_station(price_days=days, alpha_degrad_cars=0.02, name="v2g_batt_days"),
            W.user_station(price_days=W.price_day_table(3, seed=6), name="users_days"),
            W.tiny_parity_station()]


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def ec_of(counts):
    return np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(counts)])


def test_mixed_launch_three_days(cxm, oracle_lib):
    """Three episodes (each with its own price day), four classes in one launch."""
    o = oracle_lib
    specs = day_classes()
    ec = ec_of([29, 17, 23, 8])
    seed, T = 51, 3 * 288 + 20
    env = cxm.Env(specs, env_class=ec, seed=seed)
    bs = o.BatchState([o.OracleClass(s) for s in specs], ec)
    g = PY.to_np(env.rollout(T, cxm.ACT_RANDOM, cxm.OUT_FULL))
    r = o.rollout(bs, seed, T)
    flips, keep = PY.compare_rollout_flips(o, g, r, specs, ec, seed)
    assert len(flips) <= 1
    PY.compare_state(env.state_arrays(), bs, specs, ec, keep=keep)
    # the day feature changes between episodes for some env of class 0
    _, oo = PY.env_layout(specs, ec)
    do = oo[0] + 6 * specs[0].n_ports + 4
    assert len(np.unique(g["obs"][:, do])) > 1


def test_reset_observe_snapshot(cxm, oracle_lib):
    o = oracle_lib
    specs = day_classes()
    ec = ec_of([6, 5, 4, 3])
    seed = 52
    env = cxm.Env(specs, env_class=ec, seed=seed)
    env.rollout(100, cxm.ACT_RANDOM)
    obs = torch.full((env.info().obs_elems,), 5.0, device="cuda")
    env.reset(obs)                                    # new episodes begin at g = 100
    ref = np.concatenate([o.OracleClass(specs[c]).observe(o.OracleClass(specs[c]).new_state(seed, e, 100))
                          for e, c in enumerate(ec)])
    PY.compare_obs(obs.cpu().numpy()[None], ref[None], specs, ec)
    assert torch.equal(env.observe(), obs)
    bs = o.BatchState([o.OracleClass(s) for s in specs], ec)
    bs.g = 100
    g = PY.to_np(env.rollout(400, cxm.ACT_RANDOM))
    r = o.rollout(bs, seed, 400)
    flips, keep = PY.compare_rollout_flips(o, g, r, specs, ec, seed)
    assert len(flips) <= 1
    assert torch.equal(env.observe(), torch.from_numpy(g["obs"][-1]).cuda())
    snap = env.get_state()
    a = PY.to_np(env.rollout(200, cxm.ACT_RANDOM))
    env.set_state(snap)
    b = PY.to_np(env.rollout(200, cxm.ACT_RANDOM))
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_served_equals_direct(cxm):
    specs = day_classes()
    reqs = [(specs[0], 200, 600, 61), (specs[1], 64, 300, 62)]
    srv = cxm.Server(2 << 30, chunk_steps=40)
    ts = [srv.submit(s, n, T, seed, cxm.OUT_FULL) for (s, n, T, seed) in reqs]
    for t, (s, n, T, seed) in zip(ts, reqs):
        got = srv.fetch(srv.wait(t), cxm.OUT_FULL, s)
        ref = PY.to_np(cxm.Env(s, n_envs=n, seed=seed).rollout(T, cxm.ACT_RANDOM, cxm.OUT_FULL))
        for k in got:
            assert np.array_equal(got[k], ref[k]), (t, k)
        srv.release(t)
    srv.close()


def test_full_size_sampled(cxm, oracle_lib):
    """65,536 stations of the table-driven station x 288 steps; 48 replayed."""
    o = oracle_lib
    spec = W.exo_station()
    n, T, seed = 65536, 288, 5
    env = cxm.Env(spec, n_envs=n, seed=seed)
    out = env.rollout(T, cxm.ACT_RANDOM)
    rng = np.random.default_rng(13)
    ids = np.unique(np.concatenate([rng.choice(n, 46, replace=False), [0, n - 1]]))
    acols = (ids[:, None] * spec.n_actions + np.arange(spec.n_actions)).ravel()
    ocols = (ids[:, None] * spec.obs_dim + np.arange(spec.obs_dim)).ravel()
    g = {"actions": out["actions"][:, torch.from_numpy(acols).cuda()].cpu().numpy(),
         "reward": out["reward"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "done": out["done"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "obs": out["obs"][:, torch.from_numpy(ocols).cuda()].cpu().numpy()}
    ec = np.zeros(len(ids), np.int32)
    bs = o.BatchState([o.OracleClass(spec)], ec, env_ids=ids)
    PY.compare_rollout(g, o.rollout(bs, seed, T), [spec], ec)
