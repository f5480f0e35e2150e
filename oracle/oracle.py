"""ctypes wrapper of the FP64 C oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke entry point and the benchmark's CPU-baseline leg use this
module.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcx_oracle.so")

ACT_EXTERNAL, ACT_RANDOM, ACT_MAX = 0, 1, 2
K_POIS = 24

_P_ORDER = ["dt_hours", "tau", "p_sell", "p_sell_grid", "fixed_cost", "alpha_sat", "alpha_declined",
            "price_base", "price_amp", "price_sigma", "arrival_peak", "cap_lo", "cap_hi", "soc0_lo",
            "soc0_hi", "tgt_lo", "tgt_hi", "dwell_mu", "dwell_sigma"]
_I_ORDER = ["steps_per_episode", "n_levels", "dwell_max"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "cx_oracle.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class StepInfo(C.Structure):
    _fields_ = [("reward", C.c_double), ("profit", C.c_double), ("e_net", C.c_double),
                ("e_grid", C.c_double), ("c_sat", C.c_double), ("M", C.c_int32), ("acc", C.c_int32),
                ("rej", C.c_int32), ("n_dep", C.c_int32), ("done", C.c_int32), ("n_occ", C.c_int32),
                ("e_to_grid", C.c_double), ("e_batt", C.c_double), ("c_sat1", C.c_double)]


class Exo(C.Structure):
    _fields_ = [("M", C.c_int32), ("z", C.c_double), ("p_buy", C.c_double),
                ("car_cap", C.c_double * K_POIS), ("car_soc", C.c_double * K_POIS),
                ("car_tgt", C.c_double * K_POIS), ("car_dwell", C.c_int32 * K_POIS),
                ("car_user", C.c_int32 * K_POIS), ("day", C.c_int32), ("day_next", C.c_int32),
                ("car_model", C.c_int32 * K_POIS)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        P, I = C.c_void_p, C.c_int32
        L.ox_class_new.restype = P
        L.ox_class_new.argtypes = [I, I, P, P, P, P, P, P, P, P]
        L.ox_class_free.argtypes = [P]
        L.ox_class_tables.argtypes = [P, P, P]
        L.ox_philox4x32_10.argtypes = [P, P, P]
        L.ox_u24.restype = C.c_double
        L.ox_u24.argtypes = [C.c_uint32]
        L.ox_project.argtypes = [P, P]
        L.ox_apply_actions.argtypes = [P, P, P, P, P, P, P, P]
        L.ox_draw_exo.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, I, P]
        L.ox_draw_actions.argtypes = [P, I, C.c_uint64, C.c_uint32, C.c_uint32, P, P]
        L.ox_transition.argtypes = [P] * 16
        L.ox_observe.argtypes = [P, P, P, P, P, P, P, P, P, I, I, P]
        L.ox_class_set_car_models.argtypes = [P, I, P, P]
        L.ox_class_set_price_days.argtypes = [P, I, P]
        L.ox_episode_day.restype = I
        L.ox_episode_day.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32]
        L.ox_rollout.restype = I
        L.ox_rollout.argtypes = [P, P, P, C.c_int64, C.c_uint64, P, P, I, I, P, P, P, P, P, P, P, P,
                                 P, P, P, P, P, P, P, I]
        L.ox_class_set_users.argtypes = [P, C.c_double, C.c_double, C.c_double]
        L.ox_class_set_v2g.argtypes = [P, I, P, P]
        L.ox_class_actions.restype = I
        L.ox_class_actions.argtypes = [P]
        L.ox_obs_dim.restype = I
        L.ox_obs_dim.argtypes = [P]
        L.ox_action_code.restype = I
        L.ox_action_code.argtypes = [P, I, I]
        L.ox_battery_power.restype = C.c_double
        L.ox_battery_power.argtypes = [P, C.c_double, I]
        L.ox_class_set_profiles.argtypes = [P, P, P]
        L.ox_policy.argtypes = [P, I, P, P, P, P, P, C.c_uint64, C.c_uint32, C.c_uint32, P, P, P]
        L.ox_bf16_round.restype = C.c_double
        L.ox_bf16_round.argtypes = [C.c_double]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ox_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def bf16_round(x: float) -> float:
    return lib().ox_bf16_round(float(x))


class OracleClass:
    """One station class inside the oracle (architecture + parameters + its tables)."""

    def __init__(self, spec):
        self.spec = spec
        self._keep = [
            np.ascontiguousarray(spec.node_parent, dtype=np.int32),
            np.ascontiguousarray(spec.node_limit_kw, dtype=np.float64),
            np.ascontiguousarray(spec.node_eta, dtype=np.float64),
            np.ascontiguousarray(spec.port_parent, dtype=np.int32),
            np.ascontiguousarray(spec.port_pmax_kw, dtype=np.float64),
            np.ascontiguousarray(spec.port_eta, dtype=np.float64),
            np.array([getattr(spec, k) for k in _P_ORDER], dtype=np.float64),
            np.array([getattr(spec, k) for k in _I_ORDER], dtype=np.int32),
        ]
        h = lib().ox_class_new(spec.n_ports, len(spec.node_parent), *[_ptr(a) for a in self._keep])
        if not h:
            raise ValueError("oracle rejected the station spec")
        self.h = C.c_void_p(h)
        self.n = spec.n_ports
        rate, price = getattr(spec, "arrival_rate", None), getattr(spec, "price_table", None)
        if rate is not None or price is not None:
            prof = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (rate, price)]
            for a in prof:
                if a is not None and a.shape != (spec.steps_per_episode,):
                    raise ValueError("profiles need steps_per_episode entries")
            self._keep += [a for a in prof if a is not None]
            lib().ox_class_set_profiles(self.h, _ptr(prof[0]), _ptr(prof[1]))
        if getattr(spec, "v2g", 0) or getattr(spec, "battery_kwh", 0.0) > 0.0:
            pdis = getattr(spec, "port_pdis_kw", None)
            pd = None if pdis is None else np.ascontiguousarray(pdis, dtype=np.float64)
            bp = np.array([spec.battery_kwh, spec.battery_kw, spec.battery_tau, spec.battery_soc0,
                           spec.alpha_degrad_battery, spec.alpha_degrad_cars], dtype=np.float64)
            self._keep += [a for a in (pd, bp) if a is not None]
            lib().ox_class_set_v2g(self.h, int(spec.v2g), _ptr(pd), _ptr(bp))
        if getattr(spec, "charge_sensitive_share", 0.0) > 0.0:
            lib().ox_class_set_users(self.h, float(spec.charge_sensitive_share), float(spec.alpha_sat1),
                                     float(spec.beta_sat1))
        days = getattr(spec, "price_days", None)
        if days is not None:
            d = np.ascontiguousarray(days, dtype=np.float64)
            if d.ndim != 2 or d.shape[1] != spec.steps_per_episode:
                raise ValueError("price_days needs shape [n_days][steps_per_episode]")
            self._keep.append(d)
            lib().ox_class_set_price_days(self.h, d.shape[0], _ptr(d))
        models = getattr(spec, "car_models", None)
        self.has_models = models is not None
        if models is not None:
            m = np.ascontiguousarray(models, dtype=np.float64)
            if m.ndim != 2 or m.shape[1] != 4 or not 1 <= m.shape[0] <= 8:
                raise ValueError("car_models needs shape [1..8][4]")
            dc = getattr(spec, "port_dc", None)
            dca = None if dc is None else np.ascontiguousarray(dc, dtype=np.int32)
            self._keep += [a for a in (m, dca) if a is not None]
            lib().ox_class_set_car_models(self.h, m.shape[0], _ptr(m), _ptr(dca))
        self.n_act = lib().ox_class_actions(self.h)
        self.has_battery = self.n_act > self.n

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ox_class_free(self.h)
        except Exception:
            pass

    @property
    def obs_dim(self) -> int:
        return lib().ox_obs_dim(self.h)

    def action_code(self, i: int, k: int) -> int:
        """The action byte of signed level k at action index i (n_ports = the battery)."""
        return lib().ox_action_code(self.h, i, k)

    def battery_power(self, soc_b: float, kb: int) -> float:
        return lib().ox_battery_power(self.h, float(soc_b), int(kb))

    def episode_day(self, seed: int, env: int, g0: int) -> int:
        """Price day of the episode that starts at global step g0 (-1 without days)."""
        return lib().ox_episode_day(self.h, seed, env, g0)

    def new_state(self, seed: int = 0, env: int = 0, g: int = 0) -> "EnvState":
        """An empty station at t_day 0 (battery at its initial SoC; its episode's
        price day drawn for (seed, env, g))."""
        st = EnvState(self.n, self.spec.battery_soc0 if self.has_battery else 0.0)
        st.day = self.episode_day(seed, env, g)
        return st

    def tables(self):
        tp = np.zeros((self.spec.steps_per_episode, K_POIS), dtype=np.uint32)
        td = np.zeros(self.spec.dwell_max, dtype=np.uint32)
        lib().ox_class_tables(self.h, _ptr(tp), _ptr(td))
        return tp, td

    def project(self, P) -> np.ndarray:
        P = np.array(P, dtype=np.float64)
        lib().ox_project(self.h, _ptr(P))
        return P

    def apply_actions(self, dwell, soc, cap, k, user=None, rbar=None) -> np.ndarray:
        d = np.ascontiguousarray(dwell, dtype=np.int32)
        u = None if user is None else np.ascontiguousarray(user, dtype=np.int32)
        rb = None if rbar is None else np.ascontiguousarray(rbar, dtype=np.float64)
        s = np.ascontiguousarray(soc, dtype=np.float64)
        c = np.ascontiguousarray(cap, dtype=np.float64)
        kk = np.ascontiguousarray(k, dtype=np.int32)
        P = np.zeros(self.n, dtype=np.float64)
        lib().ox_apply_actions(self.h, _ptr(d), _ptr(u), _ptr(s), _ptr(c), _ptr(rb), _ptr(kk), _ptr(P))
        return P

    def draw_exo(self, seed: int, env: int, g: int, t_day: int) -> Exo:
        x = Exo()
        lib().ox_draw_exo(self.h, seed, env, g, t_day, C.byref(x))
        return x

    def draw_actions(self, mode: int, seed: int, env: int, g: int, ext=None) -> np.ndarray:
        """Signed levels of the ports (and the battery, last)."""
        k = np.zeros(self.n_act, dtype=np.int32)
        e = None if ext is None else np.ascontiguousarray(ext, dtype=np.uint8)
        lib().ox_draw_actions(self.h, mode, seed, env, g, _ptr(e), _ptr(k))
        return k

    def observe(self, st: "EnvState") -> np.ndarray:
        obs = np.zeros(self.obs_dim, dtype=np.float64)
        rb = st.rbar if self.has_models else None
        lib().ox_observe(self.h, _ptr(st.dwell), _ptr(st.user), _ptr(st.soc), _ptr(st.e_rem), _ptr(st.cap),
                         _ptr(rb), _ptr(st.p_last), _ptr(st.batt), st.t_day, getattr(st, "day", -1), _ptr(obs))
        return obs

    def transition(self, st: "EnvState", k, exo: Exo):
        """One step of one env, state in place; returns (StepInfo, obs, applied powers)."""
        kk = np.ascontiguousarray(k, dtype=np.int32)
        info = StepInfo()
        obs = np.zeros(self.obs_dim, dtype=np.float64)
        P = np.zeros(self.n, dtype=np.float64)
        ret = C.c_double(st.ret)
        t_day = C.c_int32(st.t_day)
        lib().ox_transition(self.h, _ptr(st.dwell), _ptr(st.user), _ptr(st.soc), _ptr(st.e_rem),
                            _ptr(st.cap), _ptr(st.rbar), _ptr(st.p_last), _ptr(st.batt), C.byref(ret), C.byref(t_day),
                            _ptr(kk), C.byref(exo),
                            C.byref(info), _ptr(obs), _ptr(P))
        st.ret = ret.value
        st.t_day = t_day.value
        st.day = exo.day_next
        return info, obs, P

    def policy(self, hidden: int, weights, obs, seed: int, env: int, g: int, with_margin: bool = False):
        """Logits and sampled levels of one observation; with_margin adds, per
        port, the gap between the best and second-best perturbed logit."""
        w1, b1, w2, b2 = [np.ascontiguousarray(w, dtype=np.uint16) for w in weights]
        o = np.ascontiguousarray(obs, dtype=np.float64)
        L = self.spec.n_levels
        logits = np.zeros(self.n * (L + 1), dtype=np.float64)
        k = np.zeros(self.n, dtype=np.int32)
        margin = np.zeros(self.n, dtype=np.float64)
        lib().ox_policy(self.h, hidden, _ptr(w1), _ptr(b1), _ptr(w2), _ptr(b2), _ptr(o), seed, env, g,
                        _ptr(logits), _ptr(k), _ptr(margin))
        return (logits, k, margin) if with_margin else (logits, k)


class EnvState:
    """Mutable state of one env (port-major arrays) for single-env tests."""

    def __init__(self, n_ports: int, battery_soc: float = 0.0):
        self.batt = np.array([battery_soc, 0.0])   # station battery: SoC, last power
        self.dwell = np.zeros(n_ports, dtype=np.int32)
        self.user = np.zeros(n_ports, dtype=np.int32)   # 1: charge-sensitive user
        self.rbar = np.zeros(n_ports)                   # the car's maximum rate (car models)
        self.soc = np.zeros(n_ports, dtype=np.float64)
        self.e_rem = np.zeros(n_ports, dtype=np.float64)
        self.cap = np.zeros(n_ports, dtype=np.float64)
        self.p_last = np.zeros(n_ports, dtype=np.float64)
        self.ret = 0.0
        self.t_day = 0
        self.day = -1        # price day of the current episode (exploring starts)

    def put_car(self, port: int, soc: float, cap: float, dwell: int, e_rem: float, user: int = 0,
                rbar: float = 0.0):
        self.dwell[port] = dwell
        self.user[port] = user
        self.rbar[port] = rbar
        self.soc[port] = soc
        self.cap[port] = cap
        self.e_rem[port] = e_rem


def exo(M: int = 0, p_buy: float = 0.25, cars=()) -> Exo:
    """Hand-built exogenous input: cars = [(cap, soc0, tgt, dwell[, user[, model]]), ...]."""
    x = Exo()
    x.M = M
    x.z = 0.0
    x.p_buy = p_buy
    x.day = x.day_next = -1
    for j, car in enumerate(cars):
        cap, soc0, tgt, dwell = car[:4]
        x.car_cap[j], x.car_soc[j], x.car_tgt[j], x.car_dwell[j] = cap, soc0, tgt, dwell
        x.car_user[j] = car[4] if len(car) > 4 else 0
        x.car_model[j] = car[5] if len(car) > 5 else -1
    return x


class BatchState:
    """State of many envs for ox_rollout (port-major, envs concatenated)."""

    def __init__(self, classes: Sequence[OracleClass], env_class: np.ndarray, env_ids=None):
        self.classes = list(classes)
        self.env_class = np.ascontiguousarray(env_class, dtype=np.int32)
        self.env_ids = None if env_ids is None else np.ascontiguousarray(env_ids, dtype=np.int64)
        ports = np.array([c.n for c in self.classes], dtype=np.int64)[self.env_class]
        self.port_off = np.concatenate([[0], np.cumsum(ports)])
        acts = np.array([c.n_act for c in self.classes], dtype=np.int64)[self.env_class]
        self.act_off = np.concatenate([[0], np.cumsum(acts)])
        obs = np.array([c.obs_dim for c in self.classes], dtype=np.int64)[self.env_class]
        self.obs_off = np.concatenate([[0], np.cumsum(obs)])
        P = int(self.port_off[-1])
        self.n_envs = len(self.env_class)
        self.total_ports = P
        self.total_act = int(self.act_off[-1])
        self.total_obs = int(self.obs_off[-1])
        soc0 = np.array([c.spec.battery_soc0 if c.has_battery else 0.0 for c in self.classes])
        self.batt = np.zeros(2 * self.n_envs)          # per env: battery SoC, last power
        self.batt[0::2] = soc0[self.env_class]
        self.dwell = np.zeros(P, dtype=np.int32)
        self.user = np.zeros(P, dtype=np.int32)
        self.rbar = np.zeros(P)
        self.soc = np.zeros(P)
        self.e_rem = np.zeros(P)
        self.cap = np.zeros(P)
        self.p_last = np.zeros(P)
        self.ret = np.zeros(self.n_envs)
        self.g = 0
        self.t_day = 0


def rollout(bs: BatchState, seed: int, T: int, mode: int = ACT_RANDOM, act_in=None,
            want_obs: bool = True, want_act: bool = True, want_info: bool = False,
            n_threads: int = 0, out=None):
    """Run T steps of every env; returns dict of outputs (obs, act, reward, done, info).
    out: the dict of an earlier call with the same T and envs, whose arrays are
    overwritten instead of allocated."""
    if n_threads <= 0:
        n_threads = max(1, min(16, os.cpu_count() or 1))
    handles = (C.c_void_p * len(bs.classes))(*[c.h.value for c in bs.classes])
    if out is not None:
        obs, act, rew, done = (out["obs"] if want_obs else None), (out["act"] if want_act else None), \
            out["reward"], out["done"]
        assert rew.shape == (T, bs.n_envs) and (obs is None or obs.shape == (T, bs.total_obs))
    else:
        obs = np.zeros((T, bs.total_obs)) if want_obs else None
        act = np.zeros((T, bs.total_act), dtype=np.uint8) if want_act else None
        rew = np.zeros((T, bs.n_envs))
        done = np.zeros((T, bs.n_envs), dtype=np.uint8)
    info = (StepInfo * (T * bs.n_envs))() if want_info else None
    ain = None if act_in is None else np.ascontiguousarray(act_in, dtype=np.uint8)
    g = C.c_uint32(bs.g)
    t_day = C.c_int32(bs.t_day)
    used = lib().ox_rollout(handles, _ptr(bs.env_class), _ptr(bs.env_ids), bs.n_envs, seed, C.byref(g), C.byref(t_day),
                            T, mode, _ptr(ain), _ptr(bs.dwell), _ptr(bs.user), _ptr(bs.soc), _ptr(bs.e_rem),
                            _ptr(bs.cap), _ptr(bs.rbar), _ptr(bs.p_last), _ptr(bs.batt), _ptr(bs.ret), _ptr(obs), _ptr(act),
                            _ptr(rew), _ptr(done), None if info is None else C.cast(info, C.c_void_p),
                            n_threads)
    bs.g = g.value
    bs.t_day = t_day.value
    out = {"obs": obs, "act": act, "reward": rew, "done": done, "threads": used}
    if want_info:
        arr = np.ctypeslib.as_array(info).reshape(T, bs.n_envs)
        out["info"] = {f: np.array(arr[f]) for f, _ in StepInfo._fields_}
    return out
