"""Helpers shared by the GPU parity tests: run the HIP library and the FP64
oracle on the same seeded inputs and compare them element by element.

Tolerances (FP32 library vs FP64 oracle):
  * integers (levels, done flags, occupancy, dwell, arrivals, user types) -- exact;
  * FP values: |gpu - ref| <= 1e-5 * max(|ref|, floor), with floor
      1 for SoC and observations, C (battery capacity) for e_rem,
      p_sell * L_root * dt (the largest profit of one step) for rewards/returns.

Charge-sensitive users leave when a float (the energy still wanted) reaches
zero, so the two sides may take that decision differently when it lands within
rounding of zero.  compare_rollout_flips accepts such an env from the step it
parts on -- only if the oracle, replayed step by step, shows a near-tie there --
and leaves it out from then on; the flips are counted.
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
        do = o + 6 * N + 4 + (2 if getattr(s, "has_battery", False) else 0)
        if getattr(s, "has_days", False):
            kind[do + 1] = 1                      # weekend flag
            do += 2
        if getattr(s, "has_users", False):
            kind[do:do + N] = 1
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


def snapshot_soc_erem(st):
    """SoC and the energy still wanted of every port from the snapshot's fields
    (the library keeps a car as q = 1 - SoC and u = 1 - target SoC, so the
    energy still wanted is (q - u) C); empty ports read 0."""
    occ = (st["dwell"] > 0) | (st["user"] == 1)
    soc = np.where(occ, 1.0 - st["q"], 0.0)
    e_rem = np.where(occ, (st["q"] - st["u"].astype(np.float64)) * st["cap"], 0.0)
    return soc, e_rem


def compare_state(st, bs, specs, env_class, keep=None):
    """st: Env.state_arrays(); bs: oracle BatchState.  keep: optional env mask
    (envs left out after a float-decided departure went the other way)."""
    env_class = np.asarray(env_class)
    st = dict(st)
    st["soc"], st["e_rem"] = snapshot_soc_erem(st)
    keep = np.ones(len(env_class), bool) if keep is None else np.asarray(keep, bool)
    pk = np.repeat(keep, np.diff(bs.port_off))
    assert np.array_equal(st["dwell"][pk], bs.dwell[pk]), "dwell differs"
    assert np.array_equal(st["user"][pk], bs.user[pk]), "user types differ"
    assert st["g"] == bs.g and st["t_day"] == bs.t_day
    check_close("soc", st["soc"][pk], bs.soc[pk], 1.0)
    check_close("cap", st["cap"][pk], bs.cap[pk], 1.0)
    check_close("e_rem", st["e_rem"][pk], bs.e_rem[pk], np.maximum(bs.cap[pk], 1.0))
    pmax = np.concatenate([specs[c].port_pmax_kw for c in env_class])
    check_close("p_last", st["p_last"][pk], bs.p_last[pk], pmax[pk])
    check_close("return", st["ret"][keep], bs.ret[keep], reward_floor(specs, env_class)[keep])
    has_m = np.repeat(np.array([getattr(specs[c], "car_models", None) is not None for c in env_class]) & keep,
                      np.diff(bs.port_off))
    if has_m.any():
        check_close("car rate", st["rbar"][has_m], bs.rbar[has_m], 1.0)
    has_b = np.array([specs[c].has_battery for c in env_class]) & keep
    if has_b.any():
        check_close("battery soc", st["batt_soc"][has_b], bs.batt[0::2][has_b], 1.0)
        bkw = np.array([specs[c].battery_kw for c in env_class])[has_b]
        check_close("battery power", st["batt_p"][has_b], bs.batt[1::2][has_b], bkw)


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


# ---- float-decided departures (charge-sensitive users) -----------------------

TIE_KWH = 1e-4   # |energy still wanted| below this at a departure decision is a near-tie


def env_mismatch_steps(gpu, ref, specs, env_class):
    """First step at which each env's records differ beyond tolerance (T if never)."""
    T, E = gpu["reward"].shape
    ao, oo = env_layout(specs, env_class)
    bad = np.zeros((T, E), bool)
    if "actions" in gpu and gpu["actions"] is not None and ref.get("act") is not None:
        d = gpu["actions"] != ref["act"]
        for e in range(E):
            bad[:, e] |= d[:, ao[e]:ao[e + 1]].any(axis=1)
    bad |= gpu["done"] != ref["done"]
    floor = reward_floor(specs, env_class)[None, :]
    g, r = np.asarray(gpu["reward"], np.float64), np.asarray(ref["reward"], np.float64)
    bad |= np.abs(g - r) > REL * np.maximum(np.abs(r), floor)
    if "obs" in gpu and ref.get("obs") is not None:
        kind, scale = obs_masks(specs, env_class)
        go, ro = np.asarray(gpu["obs"], np.float64), np.asarray(ref["obs"], np.float64)
        ints = kind > 0
        dint = np.zeros_like(go, dtype=bool)
        dint[:, ints] = np.rint(go[:, ints] * scale[ints]) != np.rint(ro[:, ints] * scale[ints])
        dfp = np.zeros_like(go, dtype=bool)
        dfp[:, ~ints] = np.abs(go[:, ~ints] - ro[:, ~ints]) > REL * np.maximum(np.abs(ro[:, ~ints]), 1.0)
        d = dint | dfp
        for e in range(E):
            bad[:, e] |= d[:, oo[e]:oo[e + 1]].any(axis=1)
    first = np.where(bad.any(axis=0), bad.argmax(axis=0), T)
    return first


def near_tie_steps(o, spec, seed, env_id, T, mode=1, act_in=None, g0=0):
    """Replay one env in the oracle; steps whose charge-sensitive departure test
    (energy still wanted after charging <= 0) was within TIE_KWH of zero."""
    c = o.OracleClass(spec)
    st = c.new_state(seed, env_id, g0)
    ties = []
    for t in range(T):
        g = g0 + t
        ext = None if act_in is None else act_in[t]
        k = c.draw_actions(mode, seed, env_id, g, ext)
        x = c.draw_exo(seed, env_id, g, st.t_day)
        cs = ((st.dwell > 0) | (st.user == 1)) & (st.user == 1)
        e_before = st.e_rem.copy()
        _, _, P = c.transition(st, k, x)
        after = e_before - spec.dt_hours * P
        if np.any(np.abs(after[cs]) < TIE_KWH):
            ties.append(t)
    return ties


def compare_rollout_flips(o, gpu, ref, specs, env_class, seed, mode=1, act_in=None, lag=2):
    """compare_rollout, except that an env whose records part from the oracle's at
    step t is accepted when the oracle replay shows a near-tie at a step in
    [t - lag, t]; such envs are left out from t on.  Returns the accepted (env, t)."""
    env_class = np.asarray(env_class)
    first = env_mismatch_steps(gpu, ref, specs, env_class)
    T = gpu["reward"].shape[0]
    flips = []
    ao, _ = env_layout(specs, env_class)
    for e in np.flatnonzero(first < T):
        t = int(first[e])
        spec = specs[env_class[e]]
        ain = None if act_in is None else act_in[:, ao[e]:ao[e + 1]]
        ties = near_tie_steps(o, spec, seed, int(e), t + 1, mode, ain)
        assert any(t - lag <= s <= t for s in ties), (
            f"env {e} (class {env_class[e]}) parts from the oracle at step {t} without a near-tie "
            f"(near-ties at {ties[-5:]})")
        flips.append((int(e), t))
    keep = first == T
    if keep.any():
        ks = np.flatnonzero(keep)
        sub = {k: v[:, ks] for k, v in (("reward", gpu["reward"]), ("done", gpu["done"]))}
        rsub = {"reward": ref["reward"][:, ks], "done": ref["done"][:, ks]}
        acols = np.concatenate([np.arange(ao[e], ao[e + 1]) for e in ks])
        if "actions" in gpu:
            sub["actions"], rsub["act"] = gpu["actions"][:, acols], ref["act"][:, acols]
        compare_rollout(sub, rsub, specs, env_class[ks], check_obs=False)
    return flips, keep


# ---- full-size launches, sampled ---------------------------------------------

def sampled_columns(specs, env_class, ids):
    """Columns of the action bytes and of the observation floats of envs ``ids``."""
    ao, oo = env_layout(specs, env_class)
    acols = np.concatenate([np.arange(ao[e], ao[e + 1]) for e in ids])
    ocols = np.concatenate([np.arange(oo[e], oo[e + 1]) for e in ids])
    return acols, ocols


def subset_state(st, specs, env_class, ids):
    """The fields of a snapshot (Env.state_arrays()) for envs ``ids`` only."""
    n_ports = np.array([s.n_ports for s in specs])[np.asarray(env_class)]
    po = np.concatenate([[0], np.cumsum(n_ports)]).astype(np.int64)
    pidx = np.concatenate([np.arange(po[e], po[e + 1]) for e in ids])
    out = {}
    for k, v in st.items():
        if isinstance(v, np.ndarray) and len(v) == po[-1]:
            out[k] = v[pidx]
        elif isinstance(v, np.ndarray) and len(v) == len(env_class):
            out[k] = v[ids]
        else:
            out[k] = v
    return out


def block_edge_ids(ec, lanes_of_class, wpb, extra=(), seed=0, n_random=16):
    """Envs at the edges of every class and of its launch blocks (a block runs
    wpb waves of 64 / lanes stations): the first and last env of each class, the
    last env of its first two blocks and the first of its second and third, plus
    a few random ones."""
    ec = np.asarray(ec)
    ids = set(int(x) for x in extra)
    for c in np.unique(ec):
        env = np.flatnonzero(ec == c)
        b, n = int(env[0]), len(env)
        spb = wpb * (64 // lanes_of_class[int(c)])
        for x in (0, n - 1, spb - 1, spb, 2 * spb - 1, 2 * spb, n - spb, n - spb - 1):
            if 0 <= x < n:
                ids.add(b + x)
    rng = np.random.default_rng(seed)
    ids |= set(int(x) for x in rng.choice(len(ec), n_random, replace=False))
    return np.array(sorted(ids), np.int64)


def run_full_size_sampled(cxm, o, specs, ec_full, seed, T, workload, ids, flips=False):
    """A rollout of every env of ec_full in the launch configuration that bench.py
    times for ``workload``; envs ``ids`` (records and final state) replayed in the
    oracle.  flips: charge-sensitive users, accept near-tie departures (at most 1
    in 50 sampled envs).  Returns the library's records of the sampled envs."""
    import torch
    from paper_2507_01522_amd.launch import configure
    ec_full = np.asarray(ec_full, np.int32)
    n = len(ec_full)
    env = cxm.Env(specs, env_class=ec_full, seed=seed) if len(specs) > 1 else cxm.Env(specs[0], n_envs=n, seed=seed)
    configure(env, workload, len(specs))
    out = env.rollout(T, cxm.ACT_RANDOM)
    acols, ocols = sampled_columns(specs, ec_full, ids)
    dev = lambda a: torch.from_numpy(np.asarray(a, np.int64)).to(out["reward"].device)
    g = {"actions": out["actions"][:, dev(acols)].cpu().numpy(),
         "reward": out["reward"][:, dev(ids)].cpu().numpy(),
         "done": out["done"][:, dev(ids)].cpu().numpy(),
         "obs": out["obs"][:, dev(ocols)].cpu().numpy()}
    del out
    ec = ec_full[ids]
    bs = o.BatchState([o.OracleClass(s) for s in specs], ec, env_ids=ids)
    ref = o.rollout(bs, seed, T)
    st = subset_state(env.state_arrays(), specs, ec_full, ids)
    if flips:
        first = env_mismatch_steps(g, ref, specs, ec)
        for e in np.flatnonzero(first < T):
            ties = near_tie_steps(o, specs[ec[e]], seed, int(ids[e]), int(first[e]) + 1)
            assert any(first[e] - 2 <= s <= first[e] for s in ties), (ids[e], first[e])
        assert (first < T).sum() <= max(1, len(ids) // 50)
        compare_state(st, bs, specs, ec, keep=first >= T)
    else:
        compare_rollout(g, ref, specs, ec)
        compare_state(st, bs, specs, ec)
    return g, env
