"""The parity helpers themselves, on the CPU: the flip accounting used for
charge-sensitive users accepts identical records, and refuses a difference
that no near-tie in the oracle explains."""
import numpy as np
import pytest

import workloads as W
from tests import parity as PY


def test_flip_accounting(oracle_lib):
    o = oracle_lib
    spec = W.scale_station().replace(charge_sensitive_share=0.5, alpha_sat1=0.2, beta_sat1=0.3, arrival_peak=1.5)
    ec = np.zeros(12, np.int32)
    ref = o.rollout(o.BatchState([o.OracleClass(spec)], ec), 4, 120)
    same = {"actions": ref["act"].copy(), "reward": ref["reward"].astype(np.float32),
            "done": ref["done"].copy(), "obs": ref["obs"].astype(np.float32)}
    flips, keep = PY.compare_rollout_flips(o, same, ref, [spec], ec, 4)
    assert flips == [] and keep.all()
    bad = {k: v.copy() for k, v in same.items()}
    bad["reward"][60, 5] += 1.0
    assert PY.env_mismatch_steps(bad, ref, [spec], ec)[5] == 60
    with pytest.raises(AssertionError, match="without a near-tie"):
        PY.compare_rollout_flips(o, bad, ref, [spec], ec, 4)
