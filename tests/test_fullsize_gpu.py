"""Each workload bench.py measures, at its full size and in exactly the launch
configuration it is timed in (paper_2507_01522_amd.launch: lanes per station,
waves per block, observation stage), against the FP64 oracle on sampled
stations: the first and last station of every class, stations on both sides of
the edges of its first, second and last launch blocks, and random ones.
Records of every step (levels, rewards, done flags, observations) and the
final state of each sampled station are compared to the parity tolerances."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2507_01522_amd.launch import LAUNCH
from tests import parity as PY

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return cx


def lanes_of(cxm, specs, workload):
    lanes, wpb, _ = LAUNCH[workload]
    slots = [int(cxm.compile_layout(s)["slots"]) for s in specs]
    return [lanes if lanes is not None else min(S, 64) for S in slots], wpb


def test_uneven_full_size_sampled(cxm, oracle_lib):
    """The headline workload: 65,536 stations of the 15-class mixture (mixture
    seed 1003, env seed 3) x 288 steps, one graph launch, every class at
    min(slots, 64) lanes, 4 waves per block, 8-32-lane classes staged."""
    import bench
    specs, ec = bench.uneven_workload()
    lanes, wpb = lanes_of(cxm, specs, "uneven-batching")
    ids = PY.block_edge_ids(ec, lanes, wpb, seed=31, n_random=24)
    assert len(ids) >= 64
    print(f"uneven: {len(ec)} stations, {len(ids)} sampled", flush=True)
    g, env = PY.run_full_size_sampled(cxm, oracle_lib, specs, ec, 3, 288, "uneven-batching", ids)
    assert env.info().obs_stage == 1
    assert [env.class_info(c).lanes_per_station for c in range(len(specs))] == lanes
    assert g["done"][-1].all() and not g["done"][:-1].any()


@pytest.mark.parametrize("workload,make,seed,flips", [
    ("v2g", W.v2g_station, 3, False),
    ("users", W.user_station, 4, True),
    ("exo", W.exo_station, 5, False),
])
def test_extended_full_size_sampled(cxm, oracle_lib, workload, make, seed, flips):
    """65,536 stations x 288 steps of the V2G / charge-sensitive-user /
    table-driven workload at 8 lanes x 2 slots and 1 wave per block."""
    spec = make()
    ec = np.zeros(65536, np.int32)
    lanes, wpb = lanes_of(cxm, [spec], workload)
    ids = PY.block_edge_ids(ec, lanes, wpb, extra=range(0, 65536, 4099), seed=seed, n_random=24)
    print(f"{workload}: 65536 stations, {len(ids)} sampled", flush=True)
    g, env = PY.run_full_size_sampled(cxm, oracle_lib, [spec], ec, seed, 288, workload, ids, flips=flips)
    ci = env.class_info(0)
    assert (ci.lanes_per_station, ci.waves_per_block) == (8, 1) and ci.slots == 16


@pytest.mark.parametrize("workload,make,n,seed", [
    ("tiny", W.tiny_parity_station, 64, 1),
    ("scale", W.scale_station, 4096, 2),
])
def test_small_workloads_full(cxm, oracle_lib, workload, make, n, seed):
    """The tiny (64 stations) and scale (4,096 stations) workloads in their
    measured launch, every station replayed."""
    spec = make()
    ec = np.zeros(n, np.int32)
    ids = np.arange(n, dtype=np.int64) if n <= 64 else PY.block_edge_ids(ec, [16], 1, seed=seed, n_random=200)
    PY.run_full_size_sampled(cxm, oracle_lib, [spec], ec, seed, 288, workload, ids)
