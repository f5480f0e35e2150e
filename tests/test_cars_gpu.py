"""GPU parity of car models (AC / DC rates per car, App. A.1 car profiles) in the
extended kernels, alone and combined with V2G discharge, charge-sensitive users
and price days, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu


def car_classes():
    us = W.car_mix("us")
    return [W.exo_station(),
            W.two_charger_types().replace(v2g=1, car_models=us, port_dc=[1] * 10 + [0] * 6,
                                          alpha_degrad_cars=0.02, name="v2g_types_cars_us"),
            W.user_station(car_models=W.car_mix("europe"), port_dc=[1, 0] * 8, name="users_cars_mixed_ports"),
            W.fanout4_tree(40, 3).replace(car_models=np.array([[0.25, 50.0, 7.4, 60.0], [0.75, 70.0, 11.5, 150.0]]),
                                          name="fan40_cars_ac"),
            W.tiny_parity_station()]


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def ec_of(counts):
    return np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(counts)])


def run_checked(cxm, o, specs, ec, seed, T, mode, act_in=None):
    env = cxm.Env(specs, env_class=ec, seed=seed)
    bs = o.BatchState([o.OracleClass(s) for s in specs], ec)
    ain = None if act_in is None else torch.from_numpy(act_in).cuda()
    g = PY.to_np(env.rollout(T, mode, cxm.OUT_FULL, actions=ain))
    r = o.rollout(bs, seed, T, mode=mode, act_in=act_in)
    flips, keep = PY.compare_rollout_flips(o, g, r, specs, ec, seed, mode=mode, act_in=act_in)
    assert len(flips) <= max(1, len(ec) // 50), flips
    PY.compare_state(env.state_arrays(), bs, specs, ec, keep=keep)
    return env, g


def test_mixed_launch(cxm, oracle_lib):
    specs = car_classes()
    ec = ec_of([23, 19, 17, 11, 7])
    env, g = run_checked(cxm, oracle_lib, specs, ec, 71, 320, cxm.ACT_RANDOM)
    st = env.state_arrays()
    assert len(np.unique(st["rbar"][st["rbar"] > 0])) >= 4      # several models and both port types


def test_max_and_low_levels(cxm, oracle_lib):
    specs = car_classes()[:4]
    ec = ec_of([9, 8, 7, 6])
    run_checked(cxm, oracle_lib, specs, ec, 72, 200, cxm.ACT_MAX)
    T = 150
    n_act = sum(specs[c].n_actions for c in ec)
    act = np.random.default_rng(2).integers(0, 21, size=(T, n_act), dtype=np.uint8)
    run_checked(cxm, oracle_lib, specs, ec, 73, T, cxm.ACT_EXTERNAL, act_in=act)


def test_snapshot_observe_reset(cxm):
    specs = car_classes()
    ec = ec_of([5, 4, 4, 3, 2])
    env = cxm.Env(specs, env_class=ec, seed=74)
    a = PY.to_np(env.rollout(90, cxm.ACT_RANDOM))
    assert torch.equal(env.observe(), torch.from_numpy(a["obs"][-1]).cuda())
    snap = env.get_state()
    x = PY.to_np(env.rollout(70, cxm.ACT_RANDOM))
    env.set_state(snap)
    y = PY.to_np(env.rollout(70, cxm.ACT_RANDOM))
    for k in x:
        assert np.array_equal(x[k], y[k]), k
    env.reset()
    st = env.state_arrays()
    assert (st["rbar"] == 0).all() and (st["dwell"] == 0).all()
