"""The policy rollout that allocates nothing (cx_rollout_policy_noalloc), through
the C ABI, against cx_rollout with CX_ACT_POLICY on an equal context: the same
kernels on the same inputs, so every record and the final state must be bit for
bit the same.  Two calls in a row share the GPU's fixed scratch array, the
second on a smaller context (what the first call left there must not matter);
a context needing more scratch than the fixed size is refused before any
device work."""
import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu

H = 256


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def pair(cxm, spec, weights, n, seed):
    envs = []
    for _ in range(2):
        e = cxm.Env(spec, n_envs=n, seed=seed)
        e.set_policy(H, weights)
        envs.append(e)
    return envs


@pytest.mark.parametrize("out_mode", ["full", "act_reward"])
def test_noalloc_equals_rollout_two_calls(cxm, out_mode):
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, seed=13)
    om = cxm.OUT_FULL if out_mode == "full" else cxm.OUT_ACT_REWARD
    n_big = min(40000, cxm.NOALLOC_SCRATCH_BYTES // (spec.obs_dim * 4 + spec.n_ports) - 64)
    for n, T, seed in ((n_big, 12, 81), (1000, 30, 82)):   # the second call is smaller
        print(f"noalloc {out_mode}: {n} envs x {T} steps, seed {seed}", flush=True)
        ref, na = pair(cxm, spec, weights, n, seed)
        a = PY.to_np(ref.rollout(T, cxm.ACT_POLICY, om))
        b = PY.to_np(na.rollout_policy_noalloc(T, om))
        assert set(a) == set(b)
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        assert ref.get_state() == na.get_state()
        # a second rollout continues from the state and clock the first left
        a2 = PY.to_np(ref.rollout(5, cxm.ACT_POLICY, om))
        b2 = PY.to_np(na.rollout_policy_noalloc(5, om))
        for k in a2:
            assert np.array_equal(a2[k], b2[k]), k
        del ref, na
        torch.cuda.synchronize()


def test_noalloc_refuses_beyond_scratch(cxm):
    spec = W.policy_station()
    weights = W.policy_weights(spec.n_ports, hidden=H, seed=13)
    n = cxm.NOALLOC_SCRATCH_BYTES // (spec.obs_dim * 4) + 1
    env = cxm.Env(spec, n_envs=n, seed=3)
    env.set_policy(H, weights)
    g0 = env.info().g
    with pytest.raises(cxm.CxError, match="more than the fixed"):
        env.rollout_policy_noalloc(4, cxm.OUT_ACT_REWARD)
    assert env.info().g == g0      # refused before any work: the clock did not move


def test_noalloc_needs_a_policy(cxm):
    env = cxm.Env(W.policy_station(), n_envs=8, seed=3)
    with pytest.raises(cxm.CxError, match="no policy"):
        env.rollout_policy_noalloc(4, cxm.OUT_ACT_REWARD)
