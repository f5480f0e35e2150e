"""MI355X-native batched EV charging-station simulator (the Chargax environment step).

The simulator runs in the HIP library ``libcx.so`` behind the C ABI of
``include/cx.h``; :mod:`paper_2507_01522_amd.cx` is its Python binding.
"""
from .cx import (ACT_EXTERNAL, ACT_MAX, ACT_POLICY, ACT_RANDOM, OUT_ACT_REWARD, OUT_FULL, OUT_REWARD,
                 CxError, Env, Server, lib)

__all__ = ["Env", "Server", "CxError", "lib", "ACT_EXTERNAL", "ACT_RANDOM", "ACT_MAX", "ACT_POLICY", "OUT_FULL",
           "OUT_REWARD", "OUT_ACT_REWARD"]
