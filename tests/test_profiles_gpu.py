"""GPU parity with time-of-day profiles (per-step arrival means and base
prices): commuter arrivals and a time-of-use tariff on the two-charger station,
mixed in one context with a default-profile class, and through the server."""
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


def test_profile_rollout_parity(cxm, oracle_lib):
    """Two classes (time-of-use / commuter profile and default curves), 300 steps."""
    specs = [W.profile_station(), W.scale_station()]
    ec = np.repeat([0, 1], [70, 30]).astype(np.int32)
    seed, T = 41, 300
    env = cxm.Env(specs, env_class=ec, seed=seed)
    g = PY.to_np(env.rollout(T, cxm.ACT_RANDOM, cxm.OUT_FULL))
    bs = oracle_lib.BatchState([oracle_lib.OracleClass(s) for s in specs], ec)
    ref = oracle_lib.rollout(bs, seed, T)
    PY.compare_rollout(g, ref, specs, ec)
    PY.compare_state(env.state_arrays(), bs, specs, ec)
    # the tariff is visible in the observation: base price of the peak hours
    dim = specs[0].obs_dim
    step_after = 210                      # record of step 209 observes t_day 210 (17:30)
    assert np.allclose(g["obs"][step_after - 1, 6 * 16 + 2:dim * 70:dim], specs[0].price_table[step_after])


def test_profile_request_served(cxm):
    spec = W.profile_station()
    srv = cxm.Server(2 << 30, chunk_steps=40)
    t = srv.submit(spec, 50, 290, 9, cxm.OUT_FULL)
    got = srv.fetch(srv.wait(t), cxm.OUT_FULL, spec.n_ports)
    srv.release(t)
    srv.close()
    env = cxm.Env(spec, n_envs=50, seed=9)
    ref = PY.to_np(env.rollout(290, cxm.ACT_RANDOM, cxm.OUT_FULL))
    for k in got:
        assert np.array_equal(got[k], ref[k]), k
