"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Integers bit-exact, FP within the tolerances of parity.py."""
import math

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


def run_both(cxm, o, specs, env_class, seed, T, mode, act_in=None, lanes=None, wpb=4, chunks=None):
    env_class = np.asarray(env_class, np.int32)
    if len(specs) == 1:
        env = cxm.Env(specs[0], n_envs=len(env_class), seed=seed)
    else:
        env = cxm.Env(specs, env_class=env_class, seed=seed)
    if lanes is not None:
        for c, L in enumerate(lanes):
            env.set_packing(c, L, wpb)
    classes = [o.OracleClass(s) for s in specs]
    bs = o.BatchState(classes, env_class)
    ain = None if act_in is None else torch.from_numpy(act_in).cuda()
    gout = PY.to_np(env.rollout(T, mode, cxm.OUT_FULL, actions=ain))
    ref = o.rollout(bs, seed, T, mode=mode, act_in=act_in)
    return env, bs, gout, ref


def test_tiny_parity_full(cxm, oracle_lib):
    """64 envs x 288 steps, 16 ports under 150 kW, random levels, every output."""
    specs = [W.tiny_parity_station()]
    ec = np.zeros(64, np.int32)
    env, bs, g, r = run_both(cxm, oracle_lib, specs, ec, 1, 288, cxm.ACT_RANDOM)
    PY.compare_rollout(g, r, specs, ec)
    PY.compare_state(env.state_arrays(), bs, specs, ec)
    assert g["done"][-1].all() and not g["done"][:-1].any()
    assert g["actions"].max() == 10 and g["actions"].min() == 0


def test_plain_steps_equal_persistent(cxm, oracle_lib):
    """300 one-launch steps == one 300-step persistent launch == oracle."""
    spec = W.scale_station()
    n = 200
    a = cxm.Env(spec, n_envs=n, seed=2)
    b = cxm.Env(spec, n_envs=n, seed=2)
    T = 300
    roll = PY.to_np(a.rollout(T, cxm.ACT_RANDOM))
    steps = [PY.to_np(b.step(cxm.ACT_RANDOM)) for _ in range(T)]
    plain = {k: np.concatenate([s[k] for s in steps]) for k in roll}
    for k in roll:
        assert np.array_equal(roll[k], plain[k]), k
    bs = oracle_lib.BatchState([oracle_lib.OracleClass(spec)], np.zeros(n, np.int32))
    ref = oracle_lib.rollout(bs, 2, T)
    PY.compare_rollout(plain, ref, [spec], np.zeros(n, np.int32))
    sa, sb = a.get_state(), b.get_state()
    assert sa == sb


def test_scale_parity_sampled_obs(cxm, oracle_lib):
    """4096 envs x 288 steps on the 2-level tree: every action, reward and done flag;
    observations of a sample of envs."""
    o = oracle_lib
    spec = W.scale_station()
    n, T, seed = 4096, 288, 2
    env = cxm.Env(spec, n_envs=n, seed=seed)
    out = env.rollout(T, cxm.ACT_RANDOM)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(n, 48, replace=False))
    cols = (sample[:, None] * spec.obs_dim + np.arange(spec.obs_dim)).ravel()
    g = {"actions": out["actions"].cpu().numpy(), "reward": out["reward"].cpu().numpy(),
         "done": out["done"].cpu().numpy(), "obs": out["obs"][:, torch.from_numpy(cols).cuda()].cpu().numpy()}
    bs = o.BatchState([o.OracleClass(spec)], np.zeros(n, np.int32))
    ref = o.rollout(bs, seed, T, want_obs=False)
    PY.compare_rollout(g, ref, [spec], np.zeros(n, np.int32), check_obs=False)
    bs2 = o.BatchState([o.OracleClass(spec)], np.zeros(len(sample), np.int32), env_ids=sample)
    ref2 = o.rollout(bs2, seed, T)
    PY.compare_obs(g["obs"], ref2["obs"], [spec], np.zeros(len(sample), np.int32))
    PY.compare_state(env.state_arrays(), bs, [spec], np.zeros(n, np.int32))


MIX = W.mixture_classes()


def test_all_classes_default_packing(cxm, oracle_lib):
    """Every class of the uneven mixture in one launch, ragged env counts, two days."""
    counts = [3, 9, 17, 5, 8, 11, 2, 7, 4, 6, 3, 5, 1, 2, 3]
    ec = np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(counts)])
    env, bs, g, r = run_both(cxm, oracle_lib, MIX, ec, 3, 600, cxm.ACT_RANDOM)
    PY.compare_rollout(g, r, MIX, ec)
    PY.compare_state(env.state_arrays(), bs, MIX, ec)


@pytest.mark.parametrize("ports", [8, 16, 32, 64, 128])
def test_every_packing(cxm, oracle_lib, ports):
    specs = [W.fanout4_tree(ports, d) for d in (1, 2, 3)]
    ec = np.repeat(np.arange(3, dtype=np.int32), [13, 6, 9])
    S = ports
    for L in (4, 8, 16, 32, 64):
        if S % L or S // L not in (1, 2, 4):
            continue
        for wpb in (1, 4):
            env, bs, g, r = run_both(cxm, oracle_lib, specs, ec, 4, 150, cxm.ACT_RANDOM,
                                     lanes=[L] * 3, wpb=wpb)
            PY.compare_rollout(g, r, specs, ec)
            PY.compare_state(env.state_arrays(), bs, specs, ec)


def test_external_actions_and_penalties(cxm, oracle_lib):
    """Caller-given levels (with values above 10 clamped), penalties, fixed cost,
    port efficiencies, an uneven padded tree and busy arrivals."""
    specs = [W.two_charger_types().replace(alpha_sat=0.3, alpha_declined=0.7, fixed_cost=0.05,
                                           port_eta=[0.9] * 10 + [0.95] * 6, arrival_peak=2.0),
             W.scale_station().replace(alpha_sat=0.1, alpha_declined=1.0, arrival_peak=1.5,
                                       port_eta=[0.92] * 16)]
    ec = np.repeat(np.arange(2, dtype=np.int32), [21, 30])
    T = 320
    ports = sum(specs[c].n_ports for c in ec)
    act = np.random.default_rng(5).integers(0, 14, size=(T, ports), dtype=np.uint8)
    env, bs, g, r = run_both(cxm, oracle_lib, specs, ec, 6, T, cxm.ACT_EXTERNAL, act_in=act)
    PY.compare_rollout(g, r, specs, ec)
    PY.compare_state(env.state_arrays(), bs, specs, ec)
    assert np.array_equal(g["actions"], np.minimum(act, 10))


def test_max_mode_deep_tree(cxm, oracle_lib):
    """The max-charge baseline on a 4-level tree with tight limits."""
    spec = W.fanout4_tree(64, 4, factor=0.5).replace(arrival_peak=3.0)
    ec = np.zeros(37, np.int32)
    env, bs, g, r = run_both(cxm, oracle_lib, [spec], ec, 7, 300, cxm.ACT_MAX)
    PY.compare_rollout(g, r, [spec], ec)
    PY.compare_state(env.state_arrays(), bs, [spec], ec)


def test_reset_and_snapshot(cxm, oracle_lib):
    o = oracle_lib
    spec = W.tiny_parity_station()
    n = 40
    env = cxm.Env(spec, n_envs=n, seed=8)
    env.rollout(100, cxm.ACT_RANDOM)
    snap = env.get_state()
    a = PY.to_np(env.rollout(250, cxm.ACT_RANDOM))
    env.set_state(snap)
    b1 = PY.to_np(env.rollout(90, cxm.ACT_RANDOM))
    b2 = PY.to_np(env.rollout(160, cxm.ACT_RANDOM))
    for k in a:
        assert np.array_equal(a[k], np.concatenate([b1[k], b2[k]])), k
    # reset: empty stations at t_day 0, g kept, reset observation
    obs = torch.full((1, n * spec.obs_dim), 7.0, device="cuda")
    env.reset(obs[0])
    st = env.state_arrays()
    assert st["t_day"] == 0 and st["g"] == 350 and (st["dwell"] == 0).all() and (st["ret"] == 0).all()
    ref = o.OracleClass(spec).observe(o.EnvState(spec.n_ports))
    PY.compare_obs(obs.cpu().numpy(), np.tile(ref, n)[None, :], [spec], np.zeros(n, np.int32))
    # after reset the oracle continues identically from g = 350
    bs = o.BatchState([o.OracleClass(spec)], np.zeros(n, np.int32))
    bs.g = 350
    ref2 = o.rollout(bs, 8, 300)
    g2 = PY.to_np(env.rollout(300, cxm.ACT_RANDOM))
    PY.compare_rollout(g2, ref2, [spec], np.zeros(n, np.int32))


def test_device_tables_equal_oracle(cxm, oracle_lib):
    ec = np.arange(15, dtype=np.int32)
    env = cxm.Env(MIX, env_class=ec, seed=1)
    for c in range(15):
        tp, td = env.tables(c)
        otp, otd = oracle_lib.OracleClass(MIX[c]).tables()
        assert np.array_equal(tp, otp) and np.array_equal(td[1:], otd[1:])


def test_single_env_and_zero_steps(cxm, oracle_lib):
    spec = W.fanout4_tree(128, 3)
    env, bs, g, r = run_both(cxm, oracle_lib, [spec], np.zeros(1, np.int32), 9, 301, cxm.ACT_RANDOM)
    PY.compare_rollout(g, r, [spec], np.zeros(1, np.int32))
    before = env.get_state()
    env.rollout(0, cxm.ACT_RANDOM)
    assert env.get_state() == before


def test_invalid_arguments_raise(cxm):
    env = cxm.Env(W.tiny_parity_station(), n_envs=4, seed=0)
    with pytest.raises(cxm.CxError):
        env.rollout(5, cxm.ACT_EXTERNAL)          # no actions given
    with pytest.raises(cxm.CxError):
        env.set_packing(0, 128, 4)                # more lanes than slots
    with pytest.raises(cxm.CxError):
        cxm.Env(W.tiny_parity_station().replace(tau=2.0), n_envs=4)


@pytest.mark.parametrize("kind", ["charging", "extended"])
def test_largest_station(cxm, oracle_lib, kind):
    """256 ports (the most slots a station may have: 64 lanes x 4 slots), a
    four-level tree, busy arrivals; charging-only and with V2G, a battery,
    charge-sensitive users, price days and car models."""
    o = oracle_lib
    spec = W.fanout4_tree(256, 4, factor=0.6).replace(arrival_peak=6.0, alpha_sat=0.1)
    if kind == "extended":
        spec = spec.replace(v2g=1, battery_kwh=300.0, battery_kw=100.0, charge_sensitive_share=0.4,
                            alpha_sat1=0.1, beta_sat1=0.3, price_days=W.price_day_table(5),
                            car_models=W.car_mix("us"), port_dc=[1, 0] * 128)
    ec = np.zeros(11, np.int32)
    env = cxm.Env(spec, n_envs=len(ec), seed=81)
    assert env.class_info(0).slots == 256 and env.class_info(0).lanes_per_station == 64
    bs = o.BatchState([o.OracleClass(spec)], ec)
    g = PY.to_np(env.rollout(300, cxm.ACT_RANDOM, cxm.OUT_FULL))
    r = o.rollout(bs, 81, 300)
    flips, keep = PY.compare_rollout_flips(o, g, r, [spec], ec, 81)
    assert len(flips) <= 1
    PY.compare_state(env.state_arrays(), bs, [spec], ec, keep=keep)


def dense_specs():
    """Trees that take the dense layout: the paper's default 10 DC + 6 AC station,
    5 + 2 ports, and a three-level tree (root -> [A -> (4, 3) ports, B -> 9 ports])."""
    three = W.StationSpec(16, [-1, 0, 0, 1, 1, 2], [120.0, 60.0, 90.0, 40.0, 30.0, 80.0], [1.0, 0.98, 1.0, 1.0, 0.95, 1.0],
                          [3] * 4 + [4] * 3 + [5] * 9, [22.0] * 16, [1.0] * 16, arrival_peak=1.5, name="dense3")
    return [W.two_charger_types().replace(arrival_peak=1.5, alpha_sat=0.1),
            W.StationSpec(7, [-1, 0, 0], [50.0, 30.0, 30.0], [1.0] * 3, [1] * 5 + [2] * 2, [22.0] * 7, [1.0] * 7,
                          arrival_peak=0.8, name="dense5p2"),
            three]


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_dense_layouts(cxm, oracle_lib, lanes):
    specs = dense_specs()
    for s in specs:
        lay = cxm.compile_layout(s)
        assert (lay["slot_lb"] & 0x80).any() and lay["slots"] == (8 if s.n_ports == 7 else 16)
    ec = np.repeat(np.arange(3, dtype=np.int32), [19, 13, 17])
    L = [min(lanes, cxm.compile_layout(s)["slots"]) for s in specs]
    for wpb in (1, 4):
        env, bs, g, r = run_both(cxm, oracle_lib, specs, ec, 91, 300, cxm.ACT_RANDOM, lanes=L, wpb=wpb)
        PY.compare_rollout(g, r, specs, ec)
        PY.compare_state(env.state_arrays(), bs, specs, ec)
    # the same trees as V2G classes (the extended kernels take the dense path too)
    vspecs = [s.replace(v2g=1, name=s.name + "_v2g") for s in specs]
    env, bs, g, r = run_both(cxm, oracle_lib, vspecs, ec, 92, 300, cxm.ACT_RANDOM, lanes=L)
    PY.compare_rollout(g, r, vspecs, ec)
    PY.compare_state(env.state_arrays(), bs, vspecs, ec)


def test_class_split_into_segments(cxm, oracle_lib):
    """1,100,000 stations of 256 ports: one step's observation block (6.8 GB) is
    beyond the kernels' 32-bit per-lane offsets, so the class runs as two
    segments; stations on both sides of the cut and at the ends match the
    oracle."""
    o = oracle_lib
    spec = W.fanout4_tree(256, 3).replace(arrival_peak=6.0)
    n, T, seed = 1_100_000, 2, 83
    chunk = ((1 << 32) - 1) // (4 * spec.obs_dim)
    chunk -= chunk % 64
    assert chunk < n
    env = cxm.Env(spec, n_envs=n, seed=seed)
    out = env.rollout(T, cxm.ACT_RANDOM)
    ids = np.array([0, 1, chunk - 2, chunk - 1, chunk, chunk + 1, n - 2, n - 1], np.int64)
    acols = (ids[:, None] * spec.n_actions + np.arange(spec.n_actions)).ravel()
    ocols = (ids[:, None] * spec.obs_dim + np.arange(spec.obs_dim)).ravel()
    g = {"actions": out["actions"][:, torch.from_numpy(acols).cuda()].cpu().numpy(),
         "reward": out["reward"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "done": out["done"][:, torch.from_numpy(ids).cuda()].cpu().numpy(),
         "obs": out["obs"][:, torch.from_numpy(ocols).cuda()].cpu().numpy()}
    del out
    ec = np.zeros(len(ids), np.int32)
    bs = o.BatchState([o.OracleClass(spec)], ec, env_ids=ids)
    PY.compare_rollout(g, o.rollout(bs, seed, T), [spec], ec)
