"""Oracle pins for V2G discharge and the station battery (App. A.1 "Car Profiles"
and "Endogenous state space", App. A.2 "Apply Actions", App. A.3 energy terms,
Eq. (ArchConst), Sec. 3 "Action Space").

* mirror symmetry: the discharging curve is the charging curve mirrored about
  SoC = 0.5, so a station whose every SoC is replaced by 1 - SoC, under negated
  levels, draws exactly the negated powers -- through the clip and the
  projection (which are pinned for charging elsewhere);
* hand-worked single steps: the discharge maximum binding, the mirrored curve
  binding, the stored energy binding, two-sided projection, the split of the
  grid energy into charging (1/eta) and discharging (eta) parts, the battery's
  clip, SoC update, degradation penalty and observation;
* the battery is the (N+1)-th pole: a battery-only station follows exactly the
  trajectory of a V2G port holding a car of the battery's size;
* random levels are uniform over the signed range (chi-square); external bytes
  clamp to the largest level.

Expected numbers below are closed forms worked by hand from the equations, not
outputs of the oracle.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W

TOL = 1e-12
DT = 5.0 / 60.0


def close(a, b, tol=TOL):
    return np.allclose(np.asarray(a, float), np.asarray(b, float), rtol=tol, atol=tol)


def flat(n, root_kw=150.0, **kw):
    base = dict(price_sigma=0.0, p_sell=0.45, p_sell_grid=0.25, arrival_peak=0.0,
                port_pmax_kw=[22.0] * n, port_eta=[1.0] * n)
    base.update(kw)
    return W.StationSpec(n, [-1], [root_kw], [1.0], [0] * n, **base)


def split2(splitter_kw, root_kw=200.0, **kw):
    return W.StationSpec(2, [-1, 0], [root_kw, splitter_kw], [1.0, 1.0], [1, 1], [22.0, 22.0], [1.0, 1.0],
                         price_sigma=0.0, arrival_peak=0.0, v2g=1, **kw)


# ---- mirror symmetry --------------------------------------------------------

@pytest.mark.parametrize("spec", [W.v2g_station(battery=False), W.fanout4_tree(12, 2).replace(v2g=1),
                                  W.fanout4_tree(40, 3).replace(v2g=1), W.two_charger_types().replace(v2g=1)],
                         ids=["split16", "fan12d2", "fan40d3", "two_types"])
def test_mirror_symmetry(oracle_lib, spec):
    o = oracle_lib
    c = o.OracleClass(spec)
    rng = np.random.default_rng(17)
    N, L = spec.n_ports, spec.n_levels
    caps = [h * e for h, e in zip(spec.node_limit_kw, spec.node_eta)]
    n_scaled = 0
    for trial in range(300):
        dwell = rng.integers(0, 3, N)                           # about a third of the ports empty
        soc = rng.integers(0, 1025, N) / 1024.0                 # dyadic: 1 - soc is exact
        cap = rng.uniform(5.0, 100.0, N)
        k = rng.integers(-L, L + 1, N)
        P = c.apply_actions(dwell, soc, cap, k)
        Pm = c.apply_actions(dwell, 1.0 - soc, cap, -k)
        assert np.array_equal(Pm, -P), trial
        raw = np.where(dwell > 0, np.abs(P), 0.0)
        n_scaled += int(raw.sum() > 0.0 and raw.sum() >= min(caps) * (1 - 1e-9))
    assert n_scaled > 20                                         # the projection was exercised


# ---- hand-worked single steps -------------------------------------------------

def test_discharge_maximum_and_mirrored_curve(oracle_lib):
    """Port 0: pdis = 11 kW binds (SoC 0.9 is on the flat part of the mirrored
    curve).  Port 1: pdis = 22 kW, SoC 0.1 -> the mirrored curve gives
    r_hat(1 - 0.1) = (1 - 0.9) * 22 / (1 - 0.8) = 11 kW."""
    o = oracle_lib
    spec = flat(2, v2g=1, port_pdis_kw=[11.0, 22.0], port_eta=[0.9, 0.9], alpha_degrad_cars=0.03)
    c = o.OracleClass(spec)
    st = c.new_state()
    st.put_car(0, 0.9, 50.0, 10, 5.0)
    st.put_car(1, 0.1, 50.0, 10, 40.0)
    info, obs, P = c.transition(st, [-10, -10], o.exo(0, 0.25))
    assert close(P, [-11.0, -11.0])
    e = -11.0 / 12.0                                            # energy per port this step
    assert close(st.soc, [0.9 + e / 50.0, 0.1 + e / 50.0])
    assert close(st.e_rem, [5.0 - e, 40.0 - e])
    assert close(info.e_net, 2 * e)
    assert close(info.e_to_grid, 0.9 * 2 * e) and close(info.e_grid, 0.9 * 2 * e)
    # net grid energy <= 0: the sell-to-grid price applies (App. A.3)
    profit = 0.45 * (2 * e) - 0.25 * (0.9 * 2 * e)
    assert close(info.profit, profit)
    assert close(info.reward, profit - 0.03 * (-0.9 * 2 * e))
    assert close(info.reward, -0.462)
    N = 2
    assert close(obs[5 * N:6 * N], [-0.5, -0.5])                # p_last / pmax is signed


def test_stored_energy_binds(oracle_lib):
    """SoC 0.004 of a 5 kWh battery holds 0.02 kWh = 0.24 kW for one 5-minute
    step; the mirrored curve would allow 0.004 * 22 / 0.2 = 0.44 kW."""
    o = oracle_lib
    c = o.OracleClass(flat(1, v2g=1))
    st = c.new_state()
    st.put_car(0, 0.004, 5.0, 10, 4.0)
    info, _, P = c.transition(st, [-10], o.exo(0, 0.25))
    assert close(P, [-0.24])
    assert abs(st.soc[0]) < 1e-15 and st.soc[0] >= 0.0


def test_charging_levels_unchanged_on_v2g_ports(oracle_lib):
    o = oracle_lib
    c = o.OracleClass(flat(2, v2g=1))
    P = c.apply_actions([5, 5], [0.5, 0.5], [60.0, 60.0], [5, 0])
    assert close(P, [11.0, 0.0])


@pytest.mark.parametrize("case", ["splitter", "root", "mixed"])
def test_two_sided_projection(oracle_lib, case):
    """Eq. (ArchConst) bounds the magnitude of a node's net power."""
    o = oracle_lib
    soc = [0.9, 0.9]
    k = [-10, -10]
    if case == "splitter":
        spec, want = split2(30.0), [-15.0, -15.0]               # |-44| > 30: scale 30/44
    elif case == "root":
        spec, want = split2(100.0, root_kw=20.0), [-10.0, -10.0]
    else:
        spec, want = split2(30.0), [22.0, -22.0]                # net 0: within the limit
        soc, k = [0.5, 0.9], [10, -10]
    c = o.OracleClass(spec)
    P = c.apply_actions([5, 5], soc, [60.0, 60.0], k)
    assert close(P, want)


def test_energy_split(oracle_lib):
    """One car charging 11 kW and one discharging 11 kW through ports of
    efficiency 0.9: net energy 0, grid energy 11/12 (1/0.9 - 0.9) > 0."""
    o = oracle_lib
    c = o.OracleClass(flat(2, v2g=1, port_eta=[0.9, 0.9], alpha_degrad_cars=0.03))
    st = c.new_state()
    st.put_car(0, 0.5, 60.0, 10, 30.0)
    st.put_car(1, 0.9, 60.0, 10, 6.0)
    info, _, P = c.transition(st, [5, -5], o.exo(0, 0.3))
    assert close(P, [11.0, -11.0])
    e = 11.0 / 12.0
    assert close(info.e_net, 0.0)
    assert close(info.e_to_grid, -0.9 * e)
    assert close(info.e_grid, e / 0.9 - 0.9 * e)
    assert close(info.profit, -0.3 * (e / 0.9 - 0.9 * e))        # buy price: net grid energy > 0
    assert close(info.reward, info.profit - 0.03 * 0.9 * e)


def test_battery_steps(oracle_lib):
    """A 100 kWh / 50 kW battery with its own knee tau_b = 0.6 (the cars' tau is
    0.8): flat charging at SoC 0.5, the tapered curve at 0.95
    ((1 - 0.95) 50 / 0.4 = 6.25 kW), the mirrored curve when discharging at 0.1
    ((1 - 0.9) 50 / 0.4 = 12.5 kW), with the degradation penalty."""
    o = oracle_lib
    spec = flat(1, battery_kwh=100.0, battery_kw=50.0, battery_tau=0.6, battery_soc0=0.5,
                alpha_degrad_battery=0.02)
    c = o.OracleClass(spec)
    assert c.n_act == 2 and c.obs_dim == 6 * 1 + 4 + 2
    st = c.new_state()
    assert close(st.batt, [0.5, 0.0])
    info, obs, _ = c.transition(st, [0, 10], o.exo(0, 0.25))
    assert close(st.batt, [0.5 + (50.0 / 12.0) / 100.0, 50.0])
    assert close(info.e_batt, 50.0 / 12.0) and close(info.e_grid, 50.0 / 12.0)
    assert close(info.reward, -0.25 * 50.0 / 12.0)              # charging: no degradation
    assert close(obs[6:10][2], spec.price_base + spec.price_amp * math.sin(2 * math.pi / 288))
    assert close(obs[10:12], [st.batt[0], 1.0])
    st.batt[0] = 0.95
    info, _, _ = c.transition(st, [0, 10], o.exo(0, 0.25))
    assert close(st.batt, [0.95 + 6.25 / 1200.0, 6.25])
    st.batt[0] = 0.1
    info, obs, _ = c.transition(st, [0, -10], o.exo(0, 0.25))
    eb = -12.5 / 12.0
    assert close(st.batt, [0.1 + eb / 100.0, -12.5])
    assert close(info.profit, -0.25 * eb)                        # sell-to-grid price: net grid < 0
    assert close(info.reward, -0.25 * eb - 0.02 * (-eb))
    assert close(obs[10:12], [0.1 + eb / 100.0, -0.25])


def test_battery_resets_each_day(oracle_lib):
    o = oracle_lib
    spec = flat(1, battery_kwh=80.0, battery_kw=40.0, battery_soc0=0.3)
    c = o.OracleClass(spec)
    st = c.new_state()
    for t in range(288):
        info, obs, _ = c.transition(st, [0, 7], o.exo(0, 0.25))
        assert bool(info.done) == (t == 287)
    assert close(st.batt, [0.3, 0.0]) and st.t_day == 0
    assert close(obs[10:12], [0.3, 0.0])


# ---- the battery is a pole ---------------------------------------------------

def test_battery_equals_a_v2g_port(oracle_lib):
    """Battery-only station vs. one V2G port (pmax = pdis = the battery's rate,
    efficiency 1, same tau) holding a car as large as the battery for the whole
    run: the same signed levels give the same SoC, power, reward and observed
    (SoC, power share) -- the battery is the (N+1)-th charging pole."""
    o = oracle_lib
    a_spec = flat(1, root_kw=1e4, battery_kwh=80.0, battery_kw=40.0, battery_tau=0.7, battery_soc0=0.35,
                  alpha_degrad_battery=0.02, p_sell=0.0)
    b_spec = flat(1, root_kw=1e4, v2g=1, port_pmax_kw=[40.0], tau=0.7, alpha_degrad_cars=0.02, p_sell=0.0)
    a, b = o.OracleClass(a_spec), o.OracleClass(b_spec)
    sa, sb = a.new_state(), b.new_state()
    sb.put_car(0, 0.35, 80.0, 10000, 0.0)
    rng = np.random.default_rng(5)
    seen = []
    for t in range(250):
        kb = int(rng.integers(-10, 11)) + (4 if t < 80 else -4 if t < 200 else 0)
        kb = max(-10, min(10, kb))
        p_buy = float(rng.uniform(0.1, 0.4))
        ia, oa, _ = a.transition(sa, [0, kb], o.exo(0, p_buy))
        ib, ob, _ = b.transition(sb, [kb], o.exo(0, p_buy))
        assert sa.batt[0] == sb.soc[0] and sa.batt[1] == sb.p_last[0], t
        assert ia.reward == ib.reward, t
        assert oa[10] == ob[1] and oa[11] == ob[5], t
        seen.append(sa.batt[0])
    # the walk crosses both knees (tau_b = 0.7 charging, 1 - tau_b = 0.3 discharging)
    assert min(seen) < 0.3 and max(seen) > 0.7


# ---- level draws --------------------------------------------------------------

def test_random_signed_levels_uniform(oracle_lib):
    o = oracle_lib
    spec = W.v2g_station()
    c = o.OracleClass(spec)
    N = spec.n_ports
    codes = []
    for env in range(40):
        for g in range(200):
            k = c.draw_actions(o.ACT_RANDOM, 3, env, g)
            codes.append(k + spec.n_levels)                    # ports and battery: 21 levels
    codes = np.array(codes)
    assert codes.min() == 0 and codes.max() == 20
    for cols in (slice(0, N), slice(N, N + 1)):
        cnt = np.bincount(codes[:, cols].ravel(), minlength=21)
        assert stats.chisquare(cnt).pvalue > 1e-4


def test_charging_only_class_with_battery_levels(oracle_lib):
    """A charging-only class keeps levels 0..L on its ports; its battery takes -L..L."""
    o = oracle_lib
    c = o.OracleClass(flat(2, battery_kwh=50.0, battery_kw=20.0))
    ks = np.array([c.draw_actions(o.ACT_RANDOM, 9, e, g) for e in range(20) for g in range(100)])
    assert ks[:, :2].min() == 0 and ks[:, :2].max() == 10
    assert ks[:, 2].min() == -10 and ks[:, 2].max() == 10
    assert [c.action_code(i, 0) for i in range(3)] == [0, 0, 10]
    k = c.draw_actions(o.ACT_EXTERNAL, 9, 0, 0, ext=[200, 3, 255])
    assert list(k) == [10, 3, 10]
    k = c.draw_actions(o.ACT_MAX, 9, 0, 0)
    assert list(k) == [10, 10, 10]
    v = o.OracleClass(flat(2, v2g=1))
    assert list(v.draw_actions(o.ACT_EXTERNAL, 9, 0, 0, ext=[0, 25])) == [-10, 10]


# ---- whole-rollout invariants ---------------------------------------------------

@pytest.mark.parametrize("idx", range(5))
def test_v2g_rollout_invariants(oracle_lib, idx):
    """A day and a half of random signed levels on every class of the V2G mix:
    every node's |net power| within its limit, SoCs in [0, 1], energy balance of
    cars that stay and of the battery, and the net grid energy identity."""
    o = oracle_lib
    spec = W.v2g_mixture()[idx]
    spec = spec.replace(arrival_peak=spec.arrival_peak * 3)
    c = o.OracleClass(spec)
    lv = []
    for h in range(spec.n_nodes):
        leaves = []
        for i, p in enumerate(spec.port_parent):
            a = p
            while a >= 0:
                if a == h:
                    leaves.append(i)
                    break
                a = spec.node_parent[a]
        lv.append(leaves)
    caps = [spec.node_limit_kw[h] * spec.node_eta[h] for h in range(spec.n_nodes)]
    eta = np.array(spec.port_eta)
    st = c.new_state()
    n_dis = 0
    for g in range(432):
        k = c.draw_actions(o.ACT_RANDOM, 4, 2, g)
        x = c.draw_exo(4, 2, g, st.t_day)
        d0, s0, c0, b0 = st.dwell.copy(), st.soc.copy(), st.cap.copy(), st.batt.copy()
        info, obs, P = c.transition(st, k, x)
        for h in range(spec.n_nodes):
            assert abs(P[lv[h]].sum()) <= caps[h] * (1 + 1e-12)
        e = spec.dt_hours * P
        n_dis += int((e < 0).sum())
        assert np.isclose(info.e_net, e.sum(), rtol=1e-12, atol=1e-12)
        assert np.isclose(info.e_to_grid, (eta * np.minimum(e, 0)).sum(), rtol=1e-12, atol=1e-12)
        assert np.isclose(info.e_grid, (np.maximum(e, 0) / eta).sum() + info.e_to_grid + info.e_batt,
                          rtol=1e-12, atol=1e-12)
        stay = (d0 > 0) & (st.dwell > 0) & (st.dwell == d0 - 1)
        assert np.allclose((st.soc[stay] - s0[stay]) * c0[stay], e[stay], rtol=1e-9, atol=1e-12)
        assert np.all((st.soc >= 0) & (st.soc <= 1))
        if spec.has_battery:
            assert 0.0 <= st.batt[0] <= 1.0
            if not info.done:
                assert np.isclose((st.batt[0] - b0[0]) * spec.battery_kwh, info.e_batt, rtol=1e-9, atol=1e-12)
            assert len(obs) == spec.obs_dim and obs[-2] == st.batt[0]
        else:
            assert info.e_batt == 0.0 and len(obs) == 6 * spec.n_ports + 4
    if spec.v2g:
        assert n_dis > 100
