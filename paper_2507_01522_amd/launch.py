"""Launch configuration of each measured workload: lanes per station of every
class, waves per block and the observation stage -- the fastest found on
MI355X by timing every legal choice on that workload.  bench.py times each
workload in exactly this configuration and the full-size parity tests run it,
so what is measured is what is checked."""
from __future__ import annotations

# workload -> (lanes per station, or None for every class at min(slots, 64);
#              waves per block; observation stage)
LAUNCH = {
    "uneven-batching": (None, 4, True),
    "v2g": (8, 1, False),
    "users": (8, 1, False),
    "exo": (8, 1, False),
    "tiny": (16, 1, False),
    "scale": (16, 1, False),
}
# The policy rollout of an 8-, 16- or 32-slot SIMPLE class is the fused kernel,
# whose launch is fixed (8 lanes per station, 4 waves per block, three blocks
# per CU); this packing serves the two-kernel path of the other classes and of
# the rollout that allocates nothing (8 lanes x 4 slots, 4 waves per block).
POLICY_LAUNCH = (8, 4)


def configure(env, workload: str, n_classes: int) -> None:
    """Set the packing of every class and the stage of ``env`` for ``workload``
    (a key of LAUNCH, or a description that opens with one and a colon)."""
    lanes, wpb, stage = LAUNCH[workload.split(":")[0]]
    for c in range(n_classes):
        L = lanes if lanes is not None else min(env.class_info(c).slots, 64)
        env.set_packing(c, L, wpb)
    env.set_obs_stage(stage)
