"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module describes *inputs* only -- station architectures, their parameters,
class mixtures, request streams and random policy weights.  It contains none of
the simulator's arithmetic; both the oracle and the HIP library consume what it
returns.

The paper's bundled datasets (price series, car and user profiles, traffic
levels; Table 1) are not available, so the synthetic distributions below stand
in for them:

* arrivals: Poisson with a day-shaped rate peaking at 0.3 cars per 5-minute step
  for a 16-port station (scaled by ports/16 for other sizes);
* cars: capacity U[40, 100] kWh, arrival SoC U[0.1, 0.5], target SoC U[0.7, 1.0],
  dwell lognormal(mu = ln 36 steps, sigma = 0.5);
* grid price 0.25 + 0.1 sin(2 pi t / 288) + N(0, 0.02) EUR/kWh, sell price 0.45;
* architectures as trees of splitters/transformers (Sec. 3 "EV Station Layout").
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

STEPS_PER_DAY = 288          # 24 h of 5-minute steps (Table 3)
PMAX_KW = 22.0


@dataclasses.dataclass
class StationSpec:
    """One station architecture plus its environment parameters.

    Nodes are the internal tree nodes (node 0 is the grid connection, every
    node's parent has a smaller index); ports are the leaves, listed in
    depth-first order so that every node's ports are contiguous.
    """

    n_ports: int
    node_parent: List[int]
    node_limit_kw: List[float]
    node_eta: List[float]
    port_parent: List[int]
    port_pmax_kw: List[float]
    port_eta: List[float]
    dt_hours: float = 5.0 / 60.0
    tau: float = 0.8
    p_sell: float = 0.45
    p_sell_grid: float = 0.25
    fixed_cost: float = 0.0
    alpha_sat: float = 0.0
    alpha_declined: float = 0.0
    steps_per_episode: int = STEPS_PER_DAY
    n_levels: int = 10
    price_base: float = 0.25
    price_amp: float = 0.1
    price_sigma: float = 0.02
    arrival_peak: float = 0.3
    cap_lo: float = 40.0
    cap_hi: float = 100.0
    soc0_lo: float = 0.1
    soc0_hi: float = 0.5
    tgt_lo: float = 0.7
    tgt_hi: float = 1.0
    dwell_mu: float = math.log(36.0)
    dwell_sigma: float = 0.5
    dwell_max: int = 1024
    name: str = ""
    # optional per-step profiles of the day (steps_per_episode entries each):
    # Poisson arrival means and base buying prices; None = the smooth defaults
    arrival_rate: Optional[np.ndarray] = None
    price_table: Optional[np.ndarray] = None
    # V2G: ports also discharge (levels -n_levels..n_levels, the negative ones a
    # share of port_pdis_kw, default port_pmax_kw); station battery (0 kWh = none)
    v2g: int = 0
    port_pdis_kw: Optional[List[float]] = None
    battery_kwh: float = 0.0
    battery_kw: float = 0.0
    battery_tau: float = 0.8
    battery_soc0: float = 0.5
    alpha_degrad_battery: float = 0.0
    alpha_degrad_cars: float = 0.0
    # charge-sensitive users (u = 1): share of arriving users, weight of
    # c_satisfaction,1 and its beta (weight of the hours left early)
    charge_sensitive_share: float = 0.0
    alpha_sat1: float = 0.0
    beta_sat1: float = 0.0
    # exploring starts: [n_days][steps_per_episode] base buying prices; every
    # episode draws one day (None = one price curve for every day)
    price_days: Optional[np.ndarray] = None
    # car models (App. A.1 car distribution): [n][4] rows of probability, capacity
    # kWh, AC rate kW, DC rate kW; port_dc marks DC ports (None = all AC)
    car_models: Optional[np.ndarray] = None
    port_dc: Optional[List[int]] = None

    @property
    def n_nodes(self) -> int:
        return len(self.node_parent)

    @property
    def has_battery(self) -> bool:
        return self.battery_kwh > 0.0

    @property
    def n_actions(self) -> int:
        """Action bytes per env: one per port, plus one for the battery."""
        return self.n_ports + (1 if self.has_battery else 0)

    @property
    def has_users(self) -> bool:
        """Some arriving users are charge-sensitive (u = 1)."""
        return self.charge_sensitive_share > 0.0

    @property
    def has_days(self) -> bool:
        return self.price_days is not None

    @property
    def obs_dim(self) -> int:
        return (6 * self.n_ports + 4 + (2 if self.has_battery else 0) + (2 if self.has_days else 0) +
                (self.n_ports if self.has_users else 0))

    def replace(self, **kw) -> "StationSpec":
        return dataclasses.replace(self, **kw)


def _ports(n: int, parent_of) -> Tuple[List[int], List[float], List[float]]:
    return [parent_of(p) for p in range(n)], [PMAX_KW] * n, [1.0] * n


def single_transformer(n_ports: int = 16, root_kw: float = 150.0, **kw) -> StationSpec:
    """All ports directly under one transformer (the tiny parity workload)."""
    pp, pm, pe = _ports(n_ports, lambda p: 0)
    return StationSpec(n_ports, [-1], [root_kw], [1.0], pp, pm, pe,
                       arrival_peak=0.3 * n_ports / 16.0, name=f"flat{n_ports}_{root_kw:g}kW", **kw)


def splitter_tree(n_splitters: int = 4, ports_per_splitter: int = 4, splitter_kw: float = 60.0,
                  root_kw: float = 200.0, **kw) -> StationSpec:
    """A transformer feeding equal splitters, each feeding equal ports."""
    n = n_splitters * ports_per_splitter
    parents = [-1] + [0] * n_splitters
    limits = [root_kw] + [splitter_kw] * n_splitters
    pp, pm, pe = _ports(n, lambda p: 1 + p // ports_per_splitter)
    return StationSpec(n, parents, limits, [1.0] * len(parents), pp, pm, pe,
                       arrival_peak=0.3 * n / 16.0,
                       name=f"split{n_splitters}x{ports_per_splitter}_{splitter_kw:g}_{root_kw:g}kW", **kw)


def fanout4_tree(n_ports: int, depth: int, factor: float = 0.7, **kw) -> StationSpec:
    """Class tree of the uneven-batching workload.

    ``depth`` counts internal levels (1 = a single transformer).  Ports are
    grouped four per deepest node, each higher level groups four nodes per
    parent, and the root takes whatever remains.  A node's limit is ``factor``
    times the sum of its children's maxima (port max for a port, limit for a
    node).
    """
    assert depth >= 1 and n_ports >= 1
    # level sizes from the deepest internal level up to (excluding) the root
    levels: List[int] = []
    if depth >= 2:
        levels.append(-(-n_ports // 4))
        for _ in range(depth - 2):
            levels.append(-(-levels[-1] // 4))
    # node ids: root 0, then shallowest level first so parents precede children
    parents = [-1]
    level_ids: List[List[int]] = []
    for size in reversed(levels):
        prev = level_ids[-1] if level_ids else [0]
        ids = list(range(len(parents), len(parents) + size))
        for j in range(size):
            parents.append(prev[j // 4] if level_ids else 0)
        level_ids.append(ids)
    deepest = level_ids[-1] if level_ids else [0]
    port_parent = [deepest[p // 4] if level_ids else 0 for p in range(n_ports)]
    # limits bottom-up
    limit = [0.0] * len(parents)
    child_max = [0.0] * len(parents)
    for p in range(n_ports):
        child_max[port_parent[p]] += PMAX_KW
    for ids in reversed(level_ids):
        for h in ids:
            limit[h] = factor * child_max[h]
            child_max[parents[h]] += limit[h]
    limit[0] = factor * child_max[0]
    return StationSpec(n_ports, parents, limit, [1.0] * len(parents), port_parent,
                       [PMAX_KW] * n_ports, [1.0] * n_ports,
                       arrival_peak=0.3 * n_ports / 16.0, name=f"fan4_n{n_ports}_d{depth}", **kw)


def commuter_arrivals(steps: int = STEPS_PER_DAY, morning: float = 0.9, evening: float = 0.6,
                      night: float = 0.02) -> np.ndarray:
    """Synthetic time-of-day arrival means (cars per step) with a morning and an
    evening peak over a small night floor: the shape of a workplace / commuter
    station's arrival data (the paper's data sets are not available)."""
    h = 24.0 * np.arange(steps) / steps
    bump = lambda c, w: np.exp(-0.5 * ((h - c) / w) ** 2)  # noqa: E731
    return night + morning * bump(8.5, 1.2) + evening * bump(17.5, 1.6)


def time_of_use_prices(steps: int = STEPS_PER_DAY, off_peak: float = 0.16, mid: float = 0.27,
                       peak: float = 0.41) -> np.ndarray:
    """Synthetic time-of-use tariff: off-peak 23-07 h, peak 17-21 h, mid otherwise."""
    h = 24.0 * np.arange(steps) / steps
    return np.where((h >= 23.0) | (h < 7.0), off_peak, np.where((h >= 17.0) & (h < 21.0), peak, mid))


def price_day_table(n_days: int = 28, steps: int = STEPS_PER_DAY, seed: int = 77) -> np.ndarray:
    """Synthetic price days for exploring starts: the time-of-use tariff scaled per
    day (weekends 15 % cheaper, a slow monthly swing, +-8 % daily noise) plus
    hourly noise; day d is a weekend day when d mod 7 >= 5 (the paper's price data
    are not available)."""
    rng = np.random.default_rng(seed)
    base = time_of_use_prices(steps)
    d = np.arange(n_days)
    level = (1.0 - 0.15 * (d % 7 >= 5)) * (1.0 + 0.1 * np.sin(2 * np.pi * d / 30.0)) * rng.uniform(0.92, 1.08, n_days)
    hourly = rng.normal(0.0, 0.01, (n_days, 24)).repeat(steps // 24, axis=1)
    return base[None, :] * level[:, None] + hourly


def car_mix(region: str = "europe") -> np.ndarray:
    """Synthetic car distributions (probability, capacity kWh, AC kW, DC kW) in
    place of the paper's Europe / US car data: small, compact, large and premium
    cars; the US mix leans to larger batteries and faster DC charging."""
    if region == "europe":
        return np.array([[0.30, 40.0, 7.4, 50.0], [0.35, 58.0, 11.0, 100.0],
                         [0.25, 77.0, 11.0, 150.0], [0.10, 95.0, 22.0, 250.0]])
    return np.array([[0.10, 50.0, 7.4, 60.0], [0.30, 70.0, 11.5, 150.0],
                     [0.40, 85.0, 11.5, 200.0], [0.20, 110.0, 19.2, 250.0]])


def exo_station(**kw) -> StationSpec:
    """The paper's default two-charger-type station (10 DC + 6 AC ports) driven
    by tables: commuter arrivals per step, exploring starts over 28 synthetic
    price days, and the European car mix (each car charges at its own AC or DC
    rate)."""
    s = two_charger_types().replace(name="types10dc6ac_commute_days_cars", arrival_rate=commuter_arrivals(),
                                    price_days=price_day_table(28), car_models=car_mix("europe"),
                                    port_dc=[1] * 10 + [0] * 6)
    return s.replace(**kw) if kw else s


def profile_station() -> StationSpec:
    """The two-charger-type station with commuter arrivals and a time-of-use tariff."""
    return two_charger_types().replace(name="types10dc6ac_tou", arrival_rate=commuter_arrivals(),
                                       price_table=time_of_use_prices())


def two_charger_types(n_dc: int = 10, n_ac: int = 6, dc_kw: float = 150.0, ac_kw: float = 11.5,
                      dc_split_kw: float = 800.0, ac_split_kw: float = 50.0,
                      root_kw: float = 700.0, **kw) -> StationSpec:
    """Sec. 3 / Fig. 3(b): one splitter per charger type under the grid connection."""
    n = n_dc + n_ac
    pp = [1] * n_dc + [2] * n_ac
    pm = [dc_kw] * n_dc + [ac_kw] * n_ac
    return StationSpec(n, [-1, 0, 0], [root_kw, dc_split_kw, ac_split_kw], [1.0, 1.0, 1.0], pp, pm,
                       [1.0] * n, arrival_peak=0.3 * n / 16.0, name=f"types{n_dc}dc{n_ac}ac", **kw)


def v2g_station(battery: bool = True, **kw) -> StationSpec:
    """A 16-port V2G station: 4 splitters of 60 kW x 4 bidirectional 22 kW ports
    under a 200 kW transformer, with (by default) a 200 kWh / 50 kW station
    battery; the synthetic stand-in for the paper's V2G and battery scenarios."""
    s = splitter_tree(4, 4, 60.0, 200.0).replace(v2g=1, name="v2g_split4x4" + ("_batt" if battery else ""))
    if battery:
        s = s.replace(battery_kwh=200.0, battery_kw=50.0, battery_tau=0.8, battery_soc0=0.5)
    return s.replace(**kw) if kw else s


def v2g_mixture() -> List[StationSpec]:
    """V2G classes of several shapes: flat and padded trees, uneven discharge
    maxima and efficiencies, with and without a battery, plus one charging-only
    class with a battery."""
    a = v2g_station(alpha_degrad_battery=0.02, alpha_degrad_cars=0.03, alpha_sat=0.1, alpha_declined=0.5)
    b = fanout4_tree(12, 2).replace(v2g=1, port_pdis_kw=[11.0] * 6 + [22.0] * 6,
                                    port_eta=[0.95] * 4 + [0.9] * 8, name="v2g_fan12_d2")
    c = two_charger_types().replace(v2g=1, battery_kwh=80.0, battery_kw=120.0, battery_tau=0.7,
                                    battery_soc0=0.3, alpha_degrad_cars=0.05, name="v2g_types_batt")
    d = fanout4_tree(40, 3).replace(v2g=1, name="v2g_fan40_d3")
    e = single_transformer(8, 120.0).replace(battery_kwh=60.0, battery_kw=30.0, battery_soc0=0.9,
                                             alpha_degrad_battery=0.01, name="flat8_batt")
    return [a, b, c, d, e]


def user_station(**kw) -> StationSpec:
    """The 16-port two-level station (4 splitters of 60 kW x 4 ports under
    200 kW) with half of the arriving users charge-sensitive (u = 1), c_satisfaction,1
    weighted 0.2 with beta 0.5: the synthetic stand-in for the paper's user
    profiles, for which it gives no data."""
    s = splitter_tree(4, 4, 60.0, 200.0).replace(charge_sensitive_share=0.5, alpha_sat1=0.2, beta_sat1=0.5,
                                                 name="split4x4_cs50")
    return s.replace(**kw) if kw else s


# ---- the five workloads ------------------------------------------------------

def tiny_parity_station() -> StationSpec:
    """64 envs x 288 steps; 16 ports under a 150 kW transformer."""
    return single_transformer(16, 150.0)


def scale_station() -> StationSpec:
    """4096 envs x 288 steps; 4 splitters of 60 kW x 4 ports, transformer 200 kW."""
    return splitter_tree(4, 4, 60.0, 200.0)


def policy_station() -> StationSpec:
    """32-port two-level tree: 8 splitters of 60 kW x 4 ports under 400 kW."""
    return splitter_tree(8, 4, 60.0, 400.0)


MIX_PORTS = (8, 16, 32, 64, 128)
MIX_PROBS = (0.3, 0.3, 0.2, 0.15, 0.05)
MIX_DEPTHS = (1, 2, 3)


def random_station(seed: int, max_ports: int = 64) -> StationSpec:
    """A random capacity tree for parity sweeps: 1-4 levels (root included), 1-4
    child nodes per node, 1-6 ports directly under each leaf node and 0-2 under
    inner nodes, ports listed depth-first (every node's ports contiguous; nodes
    left without a port below them are dropped); node limits 0.3-1.2x the sum
    of their children's maxima, efficiencies 0.85-1, port maxima from common
    charger ratings; a random arrival rate and level count."""
    rng = np.random.default_rng(seed)
    depth = int(rng.integers(1, 5))
    parent: List[int] = []
    children: List[List[int]] = []

    def add(p: int, d: int) -> None:
        h = len(parent)
        parent.append(p)
        children.append([])
        if p >= 0:
            children[p].append(h)
        if d + 1 < depth:
            for _ in range(int(rng.integers(1, 5))):
                add(h, d + 1)

    add(-1, 0)
    ratings = np.array([7.4, 11.0, 22.0, 50.0, 150.0])
    port_parent: List[int] = []
    pmax: List[float] = []

    def place(h: int) -> None:          # preorder: a node's own ports, then its children's
        k = int(rng.integers(1, 7)) if not children[h] else int(rng.integers(0, 3))
        for _ in range(k):
            if len(port_parent) < max_ports:
                port_parent.append(h)
                pmax.append(float(rng.choice(ratings)))
        for c in children[h]:
            place(c)

    place(0)
    below = [0] * len(parent)
    for h in port_parent:
        while h >= 0:
            below[h] += 1
            h = parent[h]
    keep = [h for h in range(len(parent)) if below[h] > 0]     # the root always has the first port
    remap = {h: i for i, h in enumerate(keep)}
    parent = [remap[parent[h]] if parent[h] >= 0 else -1 for h in keep]
    port_parent = [remap[h] for h in port_parent]
    n, H = len(port_parent), len(parent)
    # limits bottom-up: factor x the sum of the children's maxima (node limit or port maximum)
    child_max = [0.0] * H
    for i in range(n):
        child_max[port_parent[i]] += pmax[i]
    limit = [0.0] * H
    for h in reversed(range(H)):
        limit[h] = float(rng.uniform(0.3, 1.2)) * child_max[h]
        if parent[h] >= 0:
            child_max[parent[h]] += limit[h]
    return StationSpec(n, parent, limit, list(rng.uniform(0.9, 1.0, H)), port_parent, pmax,
                       list(rng.uniform(0.85, 1.0, n)), arrival_peak=float(rng.uniform(0.05, 0.3)) * n / 4.0,
                       n_levels=int(rng.choice([4, 10, 16])), alpha_sat=0.1, alpha_declined=0.2,
                       name=f"random{seed}")


def mixture_classes() -> List[StationSpec]:
    """The 15 station classes (ports x depth) of the uneven-batching workload."""
    return [fanout4_tree(n, d) for n in MIX_PORTS for d in MIX_DEPTHS]


def mixture_env_classes(n_envs: int, seed: int = 1003) -> np.ndarray:
    """Class index per env (into mixture_classes()), sorted so each class is contiguous."""
    rng = np.random.default_rng(seed)
    size_idx = rng.choice(len(MIX_PORTS), size=n_envs, p=MIX_PROBS)
    depth_idx = rng.integers(0, len(MIX_DEPTHS), size=n_envs)
    cls = (size_idx * len(MIX_DEPTHS) + depth_idx).astype(np.int32)
    return np.sort(cls, kind="stable")


def compact_classes(classes: Sequence[StationSpec], env_class: np.ndarray):
    """Drop classes no env uses; returns (used classes, remapped env_class)."""
    used = sorted(set(int(c) for c in np.unique(env_class)))
    remap = {c: i for i, c in enumerate(used)}
    return [classes[c] for c in used], np.array([remap[int(c)] for c in env_class], dtype=np.int32)


# ---- serving request stream ----------------------------------------------------

@dataclasses.dataclass
class Request:
    arrival_s: float
    class_index: int
    n_envs: int
    horizon: int
    seed: int


def request_stream(n: int, rate_per_s: float, seed: int = 2000,
                   horizons: Sequence[int] = (96, 288, 2016),
                   env_lo: int = 64, env_hi: int = 8192) -> List[Request]:
    """Poisson arrivals; n_envs log-uniform in [env_lo, env_hi]; horizon uniform over
    ``horizons``; station class from the uneven-batching mixture."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        size_idx = rng.choice(len(MIX_PORTS), p=MIX_PROBS)
        depth_idx = rng.integers(0, len(MIX_DEPTHS))
        n_envs = int(round(math.exp(rng.uniform(math.log(env_lo), math.log(env_hi)))))
        out.append(Request(t, int(size_idx * len(MIX_DEPTHS) + depth_idx), n_envs,
                           int(rng.choice(horizons)), int((seed * 1000003 + i) & 0xFFFFFFFFFFFF)))
    return out


# ---- policy weights -----------------------------------------------------------

def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to BF16 (nearest-even) and return the uint16 bit patterns."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def policy_weights(n_ports: int, hidden: int = 256, n_levels: int = 10, std: float = 0.02,
                   seed: int = 5):
    """Random-init MLP weights N(0, std) drawn in FP64, returned as BF16 bits:
    W1 [obs_dim][hidden], b1 [hidden], W2 [hidden][n_ports*(n_levels+1)], b2."""
    rng = np.random.default_rng(seed)
    d_in = 6 * n_ports + 4
    d_out = n_ports * (n_levels + 1)
    w1 = rng.normal(0.0, std, size=(d_in, hidden))
    b1 = rng.normal(0.0, std, size=hidden)
    w2 = rng.normal(0.0, std, size=(hidden, d_out))
    b2 = rng.normal(0.0, std, size=d_out)
    return bf16_bits(w1), bf16_bits(b1), bf16_bits(w2), bf16_bits(b2)
