"""Thin Python binding of the cx C ABI (include/cx.h).

Argument marshalling only: every step of the simulator runs in the HIP library
libcx.so.  PyTorch provides device memory (tensors) and streams.  There is no
CPU fallback -- if the library cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcx.so")

CX_OK = 0
ACT_EXTERNAL, ACT_RANDOM, ACT_MAX, ACT_POLICY = 0, 1, 2, 3
OUT_FULL, OUT_REWARD, OUT_ACT_REWARD = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 33554432   # CX_NOALLOC_SCRATCH_BYTES of include/cx.h
STATUS_NAMES = {0: "CX_OK", -1: "CX_E_INVALID", -2: "CX_E_OOM", -3: "CX_E_DEVICE", -4: "CX_E_BUSY",
                -5: "CX_E_BUDGET", -6: "CX_E_CANCELLED", -7: "CX_E_NOTFOUND"}


class CxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class StationSpecC(C.Structure):
    _fields_ = [("n_ports", C.c_int32), ("n_nodes", C.c_int32), ("node_parent", C.c_void_p),
                ("node_limit_kw", C.c_void_p), ("node_eta", C.c_void_p), ("port_parent", C.c_void_p),
                ("port_pmax_kw", C.c_void_p), ("port_eta", C.c_void_p), ("dt_hours", C.c_double),
                ("tau", C.c_double), ("p_sell", C.c_double), ("p_sell_grid", C.c_double),
                ("fixed_cost", C.c_double), ("alpha_sat", C.c_double), ("alpha_declined", C.c_double),
                ("steps_per_episode", C.c_int32), ("n_levels", C.c_int32), ("price_base", C.c_double),
                ("price_amp", C.c_double), ("price_sigma", C.c_double), ("arrival_peak", C.c_double),
                ("cap_lo", C.c_double), ("cap_hi", C.c_double), ("soc0_lo", C.c_double),
                ("soc0_hi", C.c_double), ("tgt_lo", C.c_double), ("tgt_hi", C.c_double),
                ("dwell_mu", C.c_double), ("dwell_sigma", C.c_double), ("dwell_max", C.c_int32),
                ("arrival_rate", C.c_void_p), ("price_table", C.c_void_p), ("v2g", C.c_int32),
                ("port_pdis_kw", C.c_void_p), ("battery_kwh", C.c_double), ("battery_kw", C.c_double),
                ("battery_tau", C.c_double), ("battery_soc0", C.c_double),
                ("alpha_degrad_battery", C.c_double), ("alpha_degrad_cars", C.c_double),
                ("charge_sensitive_share", C.c_double), ("alpha_sat1", C.c_double), ("beta_sat1", C.c_double),
                ("n_price_days", C.c_int32), ("price_days", C.c_void_p), ("n_car_models", C.c_int32),
                ("car_models", C.c_void_p), ("port_dc", C.c_void_p)]


class TrajC(C.Structure):
    _fields_ = [("obs", C.c_void_p), ("actions", C.c_void_p), ("reward", C.c_void_p), ("done", C.c_void_p)]


class InfoC(C.Structure):
    _fields_ = [("n_envs", C.c_int64), ("total_ports", C.c_int64), ("obs_elems", C.c_int64),
                ("n_classes", C.c_int32), ("steps_per_episode", C.c_int32), ("g", C.c_uint32),
                ("t_day", C.c_int32), ("seed", C.c_uint64), ("state_bytes", C.c_size_t),
                ("device_bytes", C.c_int64), ("obs_stage", C.c_int32)]


class ClassInfoC(C.Structure):
    _fields_ = [("env_begin", C.c_int64), ("n_envs", C.c_int64), ("port_offset", C.c_int64),
                ("obs_offset", C.c_int64), ("n_ports", C.c_int32), ("obs_dim", C.c_int32),
                ("slots", C.c_int32), ("levels", C.c_int32), ("lanes_per_station", C.c_int32),
                ("waves_per_block", C.c_int32), ("n_actions", C.c_int32)]


class ServerOptsC(C.Structure):
    _fields_ = [("chunk_steps", C.c_int32), ("max_active", C.c_int32), ("waves_per_block", C.c_int32),
                ("simulate_ns", C.c_int32)]


class RequestC(C.Structure):
    _fields_ = [("spec", StationSpecC), ("n_envs", C.c_int64), ("T", C.c_int32), ("seed", C.c_uint64),
                ("out_mode", C.c_int32), ("act_mode", C.c_int32), ("out", TrajC)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_envs", C.c_int64), ("T", C.c_int32), ("traj", TrajC),
                ("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("bytes", C.c_int64)]


EXPORTS = ["cx_create", "cx_create_multi", "cx_set_stream", "cx_get_info", "cx_get_class_info", "cx_reset",
           "cx_step", "cx_step_ex", "cx_rollout", "cx_set_policy", "cx_policy_logits", "cx_policy_sample", "cx_observe",
           "cx_get_state",
           "cx_set_state", "cx_get_tables", "cx_set_packing", "cx_set_obs_stage", "cx_autotune", "cx_synchronize",
           "cx_last_error", "cx_destroy", "cx_server_create", "cx_submit", "cx_poll", "cx_wait",
           "cx_cancel", "cx_release", "cx_server_stats", "cx_server_destroy", "cx_compile_layout",
           "cx_build_tables", "cx_rollout_policy_noalloc"]

_lib = None


def lib() -> C.CDLL:
    """Load libcx.so (building it first only if it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "cx_create": [P, I64, U64, P], "cx_create_multi": [P, I32, P, I64, U64, P],
        "cx_set_stream": [P, P], "cx_get_info": [P, P], "cx_get_class_info": [P, I32, P],
        "cx_reset": [P, P], "cx_step": [P, P, P, P, P], "cx_step_ex": [P, I32, P, P],
        "cx_rollout": [P, I32, I32, I32, P, P], "cx_set_policy": [P, I32, P, P, P, P],
        "cx_policy_logits": [P, P, I64, P], "cx_policy_sample": [P, P, I64, C.c_uint32, P],
        "cx_observe": [P, P], "cx_get_state": [P, P, C.c_size_t],
        "cx_set_state": [P, P, C.c_size_t], "cx_get_tables": [P, I32, P, P],
        "cx_set_packing": [P, I32, I32, I32], "cx_set_obs_stage": [P, I32], "cx_autotune": [P, I32, C.c_char_p],
        "cx_synchronize": [P], "cx_last_error": [], "cx_destroy": [P],
        "cx_server_create": [C.c_size_t, P, P], "cx_submit": [P, P, P], "cx_poll": [P, U64, P],
        "cx_wait": [P, U64, P], "cx_cancel": [P, U64], "cx_release": [P, U64],
        "cx_server_stats": [P, P, P, P, P], "cx_server_destroy": [P],
        "cx_compile_layout": [P, P, P, P, P, P], "cx_build_tables": [P, P, P],
        "cx_rollout_policy_noalloc": [P, I32, I32, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.cx_last_error.restype = C.c_char_p
    L.cx_destroy.restype = None
    L.cx_server_destroy.restype = None
    _lib = L
    return L


def check(st: int):
    if st != CX_OK:
        raise CxError(st, lib().cx_last_error().decode(errors="replace"))


_hip = None


def _hip_copy_to_host(dst: np.ndarray, src_ptr):
    """Synchronous device-to-host copy of a raw device pointer (server-owned buffers)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    if not src_ptr:
        raise CxError(-1, "record not produced by this request")
    st = _hip.hipMemcpy(dst.ctypes.data, src_ptr, dst.nbytes, 2)  # hipMemcpyDeviceToHost
    if st != 0:
        raise CxError(-3, f"hipMemcpy failed ({st})")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class _SpecHolder:
    """Keeps the numpy arrays of a spec alive while the C struct points at them."""

    def __init__(self, spec):
        self.arrays = [np.ascontiguousarray(spec.node_parent, np.int32),
                       np.ascontiguousarray(spec.node_limit_kw, np.float64),
                       np.ascontiguousarray(spec.node_eta, np.float64),
                       np.ascontiguousarray(spec.port_parent, np.int32),
                       np.ascontiguousarray(spec.port_pmax_kw, np.float64),
                       np.ascontiguousarray(spec.port_eta, np.float64)]
        self.profiles = [None if getattr(spec, k, None) is None else
                         np.ascontiguousarray(getattr(spec, k), np.float64) for k in ("arrival_rate", "price_table")]
        for arr in self.profiles:
            if arr is not None and arr.shape != (spec.steps_per_episode,):
                raise ValueError("arrival_rate / price_table need steps_per_episode entries")
        days = getattr(spec, "price_days", None)
        self.days = None if days is None else np.ascontiguousarray(days, np.float64)
        if self.days is not None and (self.days.ndim != 2 or self.days.shape[1] != spec.steps_per_episode):
            raise ValueError("price_days needs shape [n_days][steps_per_episode]")
        models = getattr(spec, "car_models", None)
        self.models = None if models is None else np.ascontiguousarray(models, np.float64)
        if self.models is not None and (self.models.ndim != 2 or self.models.shape[1] != 4):
            raise ValueError("car_models needs shape [n][4]")
        dc = getattr(spec, "port_dc", None)
        self.port_dc = None if dc is None else np.ascontiguousarray(dc, np.int32)
        pdis = getattr(spec, "port_pdis_kw", None)
        self.pdis = None if pdis is None else np.ascontiguousarray(pdis, np.float64)
        if self.pdis is not None and self.pdis.shape != (spec.n_ports,):
            raise ValueError("port_pdis_kw needs n_ports entries")
        a = self.arrays
        self.c = StationSpecC(spec.n_ports, len(spec.node_parent), a[0].ctypes.data, a[1].ctypes.data,
                              a[2].ctypes.data, a[3].ctypes.data, a[4].ctypes.data, a[5].ctypes.data,
                              spec.dt_hours, spec.tau, spec.p_sell, spec.p_sell_grid, spec.fixed_cost,
                              spec.alpha_sat, spec.alpha_declined, spec.steps_per_episode, spec.n_levels,
                              spec.price_base, spec.price_amp, spec.price_sigma, spec.arrival_peak,
                              spec.cap_lo, spec.cap_hi, spec.soc0_lo, spec.soc0_hi, spec.tgt_lo, spec.tgt_hi,
                              spec.dwell_mu, spec.dwell_sigma, spec.dwell_max,
                              *[None if arr is None else arr.ctypes.data for arr in self.profiles],
                              int(getattr(spec, "v2g", 0)),
                              None if self.pdis is None else self.pdis.ctypes.data,
                              float(getattr(spec, "battery_kwh", 0.0)), float(getattr(spec, "battery_kw", 0.0)),
                              float(getattr(spec, "battery_tau", 0.8)), float(getattr(spec, "battery_soc0", 0.5)),
                              float(getattr(spec, "alpha_degrad_battery", 0.0)),
                              float(getattr(spec, "alpha_degrad_cars", 0.0)),
                              float(getattr(spec, "charge_sensitive_share", 0.0)),
                              float(getattr(spec, "alpha_sat1", 0.0)), float(getattr(spec, "beta_sat1", 0.0)),
                              0 if self.days is None else self.days.shape[0],
                              None if self.days is None else self.days.ctypes.data,
                              0 if self.models is None else self.models.shape[0],
                              None if self.models is None else self.models.ctypes.data,
                              None if self.port_dc is None else self.port_dc.ctypes.data)


def compile_layout(spec) -> Dict[str, np.ndarray]:
    """Host-only: the aligned slot layout the kernels use for ``spec``."""
    h = _SpecHolder(spec)
    S, D = C.c_int32(), C.c_int32()
    port = np.zeros(256, np.int32)
    lb = np.zeros(256, np.uint32)
    cap = np.zeros((4, 256), np.float32)
    check(lib().cx_compile_layout(C.byref(h.c), C.byref(S), C.byref(D), port.ctypes.data, lb.ctypes.data,
                                  cap.ctypes.data))
    return {"slots": S.value, "levels": D.value, "slot_port": port[:S.value],
            "slot_lb": lb[:S.value], "slot_cap": cap[:D.value, :S.value]}


def build_tables(spec):
    """Host-only: the library's integer sampling tables for ``spec``."""
    h = _SpecHolder(spec)
    tp = np.zeros((spec.steps_per_episode, 24), np.uint32)
    td = np.zeros(spec.dwell_max, np.uint32)
    check(lib().cx_build_tables(C.byref(h.c), tp.ctypes.data, td.ctypes.data))
    return tp, td


class Env:
    """A batch of stations on the current HIP device (a cx_ctx)."""

    def __init__(self, specs, n_envs: Optional[int] = None, env_class: Optional[np.ndarray] = None,
                 seed: int = 0, device: str = "cuda:0"):
        if not torch.cuda.is_available():
            raise CxError(-3, "no HIP device visible to torch")
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        L = lib()
        if not isinstance(specs, (list, tuple)):
            specs = [specs]
        self.specs = list(specs)
        holders = [_SpecHolder(s) for s in self.specs]
        arr = (StationSpecC * len(holders))(*[h.c for h in holders])
        h = C.c_void_p()
        if env_class is None:
            if len(self.specs) != 1 or n_envs is None:
                raise ValueError("give n_envs for one spec, env_class for several")
            check(L.cx_create(arr, int(n_envs), int(seed), C.byref(h)))
        else:
            ec = np.ascontiguousarray(env_class, np.int32)
            check(L.cx_create_multi(arr, len(holders), ec.ctypes.data, len(ec), int(seed), C.byref(h)))
        self.h = h
        self.seed = int(seed)
        self.set_stream(torch.cuda.current_stream(self.device))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().cx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- introspection
    def info(self) -> InfoC:
        i = InfoC()
        check(lib().cx_get_info(self.h, C.byref(i)))
        return i

    def class_info(self, cls: int) -> ClassInfoC:
        i = ClassInfoC()
        check(lib().cx_get_class_info(self.h, cls, C.byref(i)))
        return i

    @property
    def n_envs(self) -> int:
        return self.info().n_envs

    def tables(self, cls: int = 0):
        spec = self.specs[cls]
        tp = np.zeros((spec.steps_per_episode, 24), np.uint32)
        td = np.zeros(spec.dwell_max, np.uint32)
        check(lib().cx_get_tables(self.h, cls, tp.ctypes.data, td.ctypes.data))
        return tp, td

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        check(lib().cx_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def set_packing(self, cls: int, lanes: int, waves_per_block: int = 4):
        check(lib().cx_set_packing(self.h, cls, lanes, waves_per_block))

    def set_obs_stage(self, on: bool):
        """Observations through each block's LDS stage (SIMPLE classes of up
        to 32 lanes per station) or stored lane by lane; same records."""
        check(lib().cx_set_obs_stage(self.h, 1 if on else 0))

    def autotune(self, T_probe: int = 32, cache_path: Optional[str] = None):
        """cx_autotune; currently switched off in the library (raises CxError):
        set packings with set_packing and the stage with set_obs_stage."""
        check(lib().cx_autotune(self.h, T_probe, None if cache_path is None else cache_path.encode()))

    def synchronize(self):
        check(lib().cx_synchronize(self.h))

    # ---- stepping
    def alloc_traj(self, T: int, out_mode: int = OUT_FULL) -> Dict[str, torch.Tensor]:
        i = self.info()
        d = self.device
        out = {"reward": torch.empty((T, i.n_envs), dtype=torch.float32, device=d),
               "done": torch.empty((T, i.n_envs), dtype=torch.uint8, device=d)}
        if out_mode == OUT_FULL:
            out["obs"] = torch.empty((T, i.obs_elems), dtype=torch.float32, device=d)
        if out_mode in (OUT_FULL, OUT_ACT_REWARD):
            out["actions"] = torch.empty((T, i.total_ports), dtype=torch.uint8, device=d)
        return out

    @staticmethod
    def _traj(out: Dict[str, torch.Tensor]) -> TrajC:
        return TrajC(_p(out.get("obs")), _p(out.get("actions")), _p(out.get("reward")), _p(out.get("done")))

    def reset(self, obs: Optional[torch.Tensor] = None):
        check(lib().cx_reset(self.h, _p(obs)))
        return obs

    def step(self, mode: int = ACT_RANDOM, actions: Optional[torch.Tensor] = None,
             out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """One plain step (one launch).  actions: uint8 [total_ports] for ACT_EXTERNAL."""
        if out is None:
            out = self.alloc_traj(1, OUT_FULL)
        t = self._traj(out)
        check(lib().cx_step_ex(self.h, mode, _p(actions), C.byref(t)))
        return out

    def rollout(self, T: int, mode: int = ACT_RANDOM, out_mode: int = OUT_FULL,
                actions: Optional[torch.Tensor] = None,
                out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """T steps in one persistent launch.  actions: uint8 [T][total_ports] for ACT_EXTERNAL."""
        if out is None:
            out = self.alloc_traj(T, out_mode)
        t = self._traj(out)
        check(lib().cx_rollout(self.h, T, mode, out_mode, _p(actions), C.byref(t)))
        return out

    def rollout_policy_noalloc(self, T: int, out_mode: int = OUT_FULL,
                               out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """cx_rollout_policy_noalloc: a policy rollout whose per-step scratch is the
        library's fixed device array (the library allocates nothing; the output
        buffers are allocated here unless given)."""
        if out is None:
            out = self.alloc_traj(T, out_mode)
        t = self._traj(out)
        check(lib().cx_rollout_policy_noalloc(self.h, T, out_mode, C.byref(t)))
        return out

    # ---- state
    def get_state(self) -> bytes:
        n = self.info().state_bytes
        buf = (C.c_ubyte * n)()
        check(lib().cx_get_state(self.h, buf, n))
        return bytes(buf)

    def set_state(self, blob: bytes):
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        check(lib().cx_set_state(self.h, buf, len(blob)))

    def state_arrays(self) -> Dict[str, np.ndarray]:
        """The fields of get_state() as arrays, unchanged: per port (env-major port
        order) dwell, q = 1 - SoC, u = 1 - target SoC, cap, p_last, user, rbar; per
        env the return and the station battery's SoC and last power (battery
        classes; other envs read as 0); g and t_day."""
        blob = self.get_state()
        i = self.info()
        head = np.frombuffer(blob, dtype=np.uint8, count=32)
        n_ports = int(head[16:24].view(np.int64)[0])
        g = int(head[24:28].view(np.uint32)[0])
        t_day = int(head[28:32].view(np.int32)[0])
        rec = np.frombuffer(blob, dtype=np.dtype([("dwell", "<i4"), ("q", "<f8"), ("u", "<f4"),
                                                  ("cap", "<f4"), ("p_last", "<f4"), ("user", "u1"),
                                                  ("rbar", "<f4")]),
                            count=n_ports, offset=32)
        off = 32 + 29 * n_ports
        ret = np.frombuffer(blob, dtype="<f8", count=i.n_envs, offset=off)
        off += 8 * i.n_envs
        bsoc = np.zeros(i.n_envs)
        bp = np.zeros(i.n_envs, np.float32)
        for c in range(i.n_classes):
            ci = self.class_info(c)
            if ci.n_actions == ci.n_ports:
                continue
            b = np.frombuffer(blob, dtype=np.dtype([("soc", "<f8"), ("p", "<f4")]), count=ci.n_envs, offset=off)
            bsoc[ci.env_begin:ci.env_begin + ci.n_envs] = b["soc"]
            bp[ci.env_begin:ci.env_begin + ci.n_envs] = b["p"]
            off += 12 * ci.n_envs
        out = {k: np.array(rec[k]) for k in rec.dtype.names}
        out["user"] = out["user"].astype(np.int32)
        out["ret"] = np.array(ret)
        out["batt_soc"] = bsoc
        out["batt_p"] = bp
        out["g"] = g
        out["t_day"] = t_day
        return out

    # ---- policy
    def set_policy(self, hidden: int, weights):
        w1, b1, w2, b2 = [np.ascontiguousarray(w, np.uint16) for w in weights]
        check(lib().cx_set_policy(self.h, hidden, w1.ctypes.data, b1.ctypes.data, w2.ctypes.data,
                                  b2.ctypes.data))

    def observe(self, obs: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Observation of the current state (one record of the obs layout)."""
        if obs is None:
            obs = torch.empty((self.info().obs_elems,), dtype=torch.float32, device=self.device)
        check(lib().cx_observe(self.h, _p(obs)))
        return obs

    def policy_sample(self, obs: torch.Tensor, g: int, act: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Levels the policy draws for obs [n][obs_dim] at global step g."""
        n = obs.shape[0]
        if act is None:
            act = torch.empty((n, self.specs[0].n_ports), dtype=torch.uint8, device=self.device)
        check(lib().cx_policy_sample(self.h, _p(obs.contiguous()), n, int(g), _p(act)))
        return act

    def policy_logits(self, obs: torch.Tensor) -> torch.Tensor:
        spec = self.specs[0]
        n = obs.shape[0]
        logits = torch.empty((n, spec.n_ports * (spec.n_levels + 1)), dtype=torch.float32, device=self.device)
        check(lib().cx_policy_logits(self.h, _p(obs.contiguous()), n, _p(logits)))
        return logits


class Server:
    """Continuous-batching rollout server (cx_server_*): requests of differing
    station class, size and horizon share every launch; results are identical
    alone or in a mix.  simulate_ns > 0 runs the scheduler on a host clock only."""

    def __init__(self, budget_bytes: int, chunk_steps: int = 144, max_active: int = 256,
                 waves_per_block: int = 4, simulate_ns: int = 0):
        if simulate_ns <= 0 and not torch.cuda.is_available():
            raise CxError(-3, "no HIP device visible to torch")
        o = ServerOptsC(chunk_steps, max_active, waves_per_block, simulate_ns)
        h = C.c_void_p()
        check(lib().cx_server_create(int(budget_bytes), C.byref(o), C.byref(h)))
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().cx_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, spec, n_envs: int, T: int, seed: int, out_mode: int = OUT_FULL,
               act_mode: int = ACT_RANDOM, out: Optional[Dict[str, torch.Tensor]] = None) -> int:
        holder = _SpecHolder(spec)
        traj = TrajC() if out is None else Env._traj(out)
        req = RequestC(holder.c, int(n_envs), int(T), int(seed), out_mode, act_mode, traj)
        t = C.c_uint64()
        check(lib().cx_submit(self.h, C.byref(req), C.byref(t)))
        self._keep[t.value] = (holder, out)
        return t.value

    def poll(self, ticket: int):
        r = ResultC()
        st = lib().cx_poll(self.h, ticket, C.byref(r))
        if st == -4:
            return None
        check(st)
        return r

    def wait(self, ticket: int) -> ResultC:
        r = ResultC()
        check(lib().cx_wait(self.h, ticket, C.byref(r)))
        return r

    def cancel(self, ticket: int):
        check(lib().cx_cancel(self.h, ticket))

    def release(self, ticket: int):
        check(lib().cx_release(self.h, ticket))
        self._keep.pop(ticket, None)

    @staticmethod
    def fetch(res: ResultC, out_mode: int, spec) -> Dict[str, np.ndarray]:
        """Copy the records of a finished request (server-owned or caller buffers)
        to host arrays shaped like Env.alloc_traj.  spec: the request's station
        spec (or, for a charging-only station, its port count)."""
        E, T = int(res.n_envs), int(res.T)
        if isinstance(spec, (int, np.integer)):
            obs_dim, n_act = 6 * int(spec) + 4, int(spec)
        else:
            obs_dim, n_act = spec.obs_dim, spec.n_actions
        want = {"reward": (np.float32, (T, E), res.traj.reward), "done": (np.uint8, (T, E), res.traj.done)}
        if out_mode == OUT_FULL:
            want["obs"] = (np.float32, (T, E * obs_dim), res.traj.obs)
        if out_mode in (OUT_FULL, OUT_ACT_REWARD):
            want["actions"] = (np.uint8, (T, E * n_act), res.traj.actions)
        out = {}
        for k, (dt, shape, ptr) in want.items():
            a = np.empty(shape, dtype=dt)
            _hip_copy_to_host(a, ptr)
            out[k] = a
        return out

    def stats(self) -> Dict[str, float]:
        b = C.c_double()
        e, n = C.c_int64(), C.c_int64()
        p = C.c_int32()
        check(lib().cx_server_stats(self.h, C.byref(b), C.byref(e), C.byref(n), C.byref(p)))
        return {"busy_s": b.value, "env_steps": e.value, "launches": n.value, "peak_active": p.value}
