"""Rollouts that write only some of their records.

Any member of cx_traj may be NULL (that record is not written).  Every proper
subset of obs / actions / reward / done, over a rollout of many steps, must
write exactly what the run with all four writes: in the staged and the
lane-store SIMPLE kernels, the general and extended kernels and the fused
policy rollout.  (A record whose pointer was NULL once shared its per-step
advance with a sibling's, so a NULL reward or done turned into a stray
address from the second step on.)"""
import itertools

import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PY

pytestmark = pytest.mark.gpu

KEYS = ("obs", "actions", "reward", "done")
SUBSETS = [s for n in (1, 2, 3) for s in itertools.combinations(KEYS, n)]
MIX = W.mixture_classes() + [W.two_charger_types(), W.v2g_station(), W.exo_station()]
COUNTS = [5, 3, 7, 9, 1, 6, 4, 11, 2, 3, 5, 1, 2, 1, 3, 6, 5, 4]
T = 40


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def mixture(cxm, stage):
    ec = np.concatenate([np.full(c, i, np.int32) for i, c in enumerate(COUNTS)])
    env = cxm.Env(MIX, env_class=ec, seed=71)
    for c, s in enumerate(MIX):
        env.set_packing(c, min(max(s.n_ports, 4), 64), 4)
    env.set_obs_stage(stage)
    return env


def policy(cxm):
    spec = W.policy_station()
    env = cxm.Env(spec, n_envs=45, seed=72)
    env.set_policy(64, W.policy_weights(spec.n_ports, hidden=64, std=0.2, seed=12))
    return env


def check_subsets(cxm, make, mode):
    ref = PY.to_np(make().rollout(T, mode, cxm.OUT_FULL))
    for sub in SUBSETS:
        env = make()
        full = env.alloc_traj(T, cxm.OUT_FULL)
        print(f"records {'+'.join(sub)}", flush=True)
        got = PY.to_np(env.rollout(T, mode, cxm.OUT_FULL, out={k: full[k] for k in sub}))
        assert sorted(got) == sorted(sub)
        for k in sub:
            assert np.array_equal(got[k], ref[k]), (sub, k)


@pytest.mark.parametrize("stage", [False, True])
def test_record_subsets_mixture(cxm, stage):
    """18 classes (SIMPLE 8-128 ports, general, V2G, table-driven), ragged counts."""
    check_subsets(cxm, lambda: mixture(cxm, stage), cxm.ACT_RANDOM)


def test_record_subsets_policy(cxm):
    """The fused policy rollout (levels from the MLP every step)."""
    check_subsets(cxm, lambda: policy(cxm), cxm.ACT_POLICY)
