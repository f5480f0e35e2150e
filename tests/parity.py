"""Helpers shared by the GPU parity tests: run the HIP library and the FP64
oracle on the same seeded inputs and compare them element by element.

Tolerances (FP32 library vs FP64 oracle):
  * integers (levels, done flags, occupancy, dwell, arrivals) -- exact;
  * FP values: |gpu - ref| <= 1e-5 * max(|ref|, floor), with floor
      1 for SoC and observations, C (battery capacity) for e_rem,
      p_sell * L_root * dt (the largest profit of one step) for rewards/returns.
"""
from __future__ import annotations

import numpy as np

REL = 1e-5


def env_layout(specs, env_class):
    """Per-env offsets of the action bytes and of the observation floats."""
    acts = np.array([s.n_actions for s in specs])[env_class]
    obs_dim = np.array([s.obs_dim for s in specs])[env_class]
    return (np.concatenate([[0], np.cumsum(acts)]).astype(np.int64),
            np.concatenate([[0], np.cumsum(obs_dim)]).astype(np.int64))


def obs_masks(specs, env_class):
    """Per obs element: kind (0 fp, 1 occupancy, 2 dwell*S, 3 n_occ*N) and integer scale."""
    _, oo = env_layout(specs, env_class)
    total = int(oo[-1])
    kind = np.zeros(total, np.int8)
    scale = np.ones(total, np.float64)
    for e, c in enumerate(env_class):
        s = specs[c]
        N, o = s.n_ports, int(oo[e])
        kind[o:o + N] = 1
        kind[o + 3 * N:o + 4 * N] = 2
        scale[o + 3 * N:o + 4 * N] = s.steps_per_episode
        kind[o + 6 * N + 3] = 3
        scale[o + 6 * N + 3] = N
    return kind, scale


def reward_floor(specs, env_class):
    """The largest profit of one step: the sell price times the root's energy
    (plus the battery's, at the larger of the buy and sell prices)."""
    f = np.array([s.p_sell * s.node_limit_kw[0] * s.node_eta[0] * s.dt_hours +
                  max(s.p_sell, s.price_base + s.price_amp) * getattr(s, "battery_kw", 0.0) * s.dt_hours
                  for s in specs])
    return f[env_class]


def check_close(name, got, ref, floor):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    bound = REL * np.maximum(np.abs(ref), floor)
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(bound, 1e-30)), err.shape)
        raise AssertionError(f"{name}: {bad.sum()} of {bad.size} beyond tolerance; worst at {i}: "
                             f"gpu={got[i]!r} ref={ref[i]!r} bound={np.broadcast_to(bound, err.shape)[i]!r}")


def compare_obs(gpu_obs, ref_obs, specs, env_class, cols=None):
    """gpu_obs/ref_obs: [T][obs_elems] (or the columns ``cols`` of it)."""
    kind, scale = obs_masks(specs, env_class)
    if cols is not None:
        kind, scale = kind[cols], scale[cols]
    g = np.asarray(gpu_obs, np.float64)
    r = np.asarray(ref_obs, np.float64)
    ints = kind > 0
    gi = np.rint(g[:, ints] * scale[ints]).astype(np.int64)
    ri = np.rint(r[:, ints] * scale[ints]).astype(np.int64)
    if not np.array_equal(gi, ri):
        t, j = np.argwhere(gi != ri)[0]
        raise AssertionError(f"integer obs mismatch at step {t} col {j}: gpu={gi[t, j]} ref={ri[t, j]}")
    check_close("obs", g[:, ~ints], r[:, ~ints], 1.0)


def compare_rollout(gpu, ref, specs, env_class, check_obs=True):
    """gpu: dict of numpy arrays from the library; ref: dict from oracle.rollout."""
    if "actions" in gpu and gpu["actions"] is not None and ref.get("act") is not None:
        a, b = gpu["actions"], ref["act"]
        if not np.array_equal(a, b):
            t, j = np.argwhere(a != b)[0]
            raise AssertionError(f"action mismatch at step {t} port {j}: gpu={a[t, j]} ref={b[t, j]}")
    assert np.array_equal(gpu["done"], ref["done"]), "done flags differ"
    check_close("reward", gpu["reward"], ref["reward"], reward_floor(specs, env_class)[None, :])
    if check_obs and "obs" in gpu:
        compare_obs(gpu["obs"], ref["obs"], specs, env_class)


def compare_state(st, bs, specs, env_class):
    """st: Env.state_arrays(); bs: oracle BatchState."""
    assert np.array_equal(st["dwell"], bs.dwell), "dwell differs"
    assert st["g"] == bs.g and st["t_day"] == bs.t_day
    check_close("soc", st["soc"], bs.soc, 1.0)
    check_close("cap", st["cap"], bs.cap, 1.0)
    check_close("e_rem", st["e_rem"], bs.e_rem, np.maximum(bs.cap, 1.0))
    pmax = np.concatenate([specs[c].port_pmax_kw for c in env_class])
    check_close("p_last", st["p_last"], bs.p_last, pmax)
    check_close("return", st["ret"], bs.ret, reward_floor(specs, env_class))
    has_b = np.array([specs[c].has_battery for c in env_class])
    if has_b.any():
        check_close("battery soc", st["batt_soc"][has_b], bs.batt[0::2][has_b], 1.0)
        bkw = np.array([specs[c].battery_kw for c in env_class])[has_b]
        check_close("battery power", st["batt_p"][has_b], bs.batt[1::2][has_b], bkw)


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}
