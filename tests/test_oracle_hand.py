"""Oracle pins: hand-worked cases, closed forms and special cases of one step.

Each expected number is worked out by hand (tests/golden/hand_cases.json) or is
a closed form of the charging dynamics; none is produced by the oracle itself.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))["cases"]
TOL = 1e-12


def two_port(o, root_kw, splitter_kw=None, eta=1.0, **kw):
    if splitter_kw is None:
        spec = W.StationSpec(2, [-1], [root_kw], [1.0], [0, 0], [22.0, 22.0], [eta, eta],
                             price_sigma=0.0, **kw)
    else:
        spec = W.StationSpec(2, [-1, 0], [root_kw, splitter_kw], [1.0, 1.0], [1, 1], [22.0, 22.0],
                             [eta, eta], price_sigma=0.0, **kw)
    return o.OracleClass(spec)


def close(a, b, tol=TOL):
    return np.allclose(np.asarray(a, float), np.asarray(b, float), rtol=tol, atol=tol)


def test_case_A_root_scaling(oracle_lib):
    o = oracle_lib
    c = two_port(o, 30.0)
    st = o.EnvState(2)
    st.put_car(0, 0.5, 60.0, 10, 20.0)
    st.put_car(1, 0.5, 60.0, 10, 20.0)
    info, obs, P = c.transition(st, [10, 10], o.exo(0, 0.25))
    g = GOLD["A_root_scaling"]
    assert close(P, g["P"]) and close(st.soc, g["soc"]) and close(st.e_rem, g["e_rem"])
    assert close(info.e_net, g["e_net"]) and close(info.e_grid, g["e_grid"])
    assert close(info.reward, g["reward"]) and close(st.ret, g["reward"])
    assert list(st.dwell) == [9, 9] and st.t_day == 1
    # observation of the new state (t' = 1): p_last / pmax = 15/22, e_rem / C = 18.75/60
    N = 2
    assert close(obs[0:N], [1, 1]) and close(obs[5 * N:6 * N], [15 / 22, 15 / 22])
    assert close(obs[2 * N:3 * N], [0.3125, 0.3125]) and close(obs[3 * N:4 * N], [9 / 288, 9 / 288])
    assert close(obs[6 * N + 3], 1.0)


def test_case_B_taper(oracle_lib):
    o = oracle_lib
    c = two_port(o, 100.0)
    st = o.EnvState(2)
    st.put_car(0, 0.9, 50.0, 10, 5.0)
    st.put_car(1, 0.5, 50.0, 10, 20.0)
    info, obs, P = c.transition(st, [10, 5], o.exo(0, 0.25))
    g = GOLD["B_taper"]
    assert close(P, g["P"]) and close(st.soc, g["soc"])
    assert close(info.e_net, g["e_net"]) and close(info.reward, g["reward"])
    assert close(obs[4 * 2:5 * 2], g["obs_rhat_over_pmax"], 1e-12)


def test_case_C_nested(oracle_lib):
    o = oracle_lib
    c = two_port(o, 20.0, splitter_kw=30.0)
    st = o.EnvState(2)
    st.put_car(0, 0.5, 60.0, 10, 20.0)
    st.put_car(1, 0.5, 60.0, 10, 20.0)
    info, obs, P = c.transition(st, [10, 10], o.exo(0, 0.25))
    g = GOLD["C_nested"]
    assert close(P, g["P"]) and close(info.e_net, g["e_net"])


def test_case_D_port_efficiency(oracle_lib):
    o = oracle_lib
    c = two_port(o, 30.0, eta=0.9)
    st = o.EnvState(2)
    st.put_car(0, 0.5, 60.0, 10, 20.0)
    st.put_car(1, 0.5, 60.0, 10, 20.0)
    info, _, _ = c.transition(st, [10, 10], o.exo(0, 0.25))
    g = GOLD["D_port_efficiency"]
    assert close(info.e_net, g["e_net"]) and close(info.e_grid, g["e_grid"])
    assert close(info.reward, g["reward"])


def test_case_E_depart_arrive(oracle_lib):
    o = oracle_lib
    spec = W.StationSpec(4, [-1], [1000.0], [1.0], [0] * 4, [22.0] * 4, [1.0] * 4, price_sigma=0.0,
                         alpha_sat=0.1, alpha_declined=0.5)
    c = o.OracleClass(spec)
    st = o.EnvState(4)
    for p in range(4):
        st.put_car(p, 0.5, 60.0, 1 if p == 2 else 5, 12.0)
    x = o.exo(3, 0.25, cars=[(50.0, 0.2, 0.8, 7), (60.0, 0.3, 0.9, 9), (70.0, 0.4, 1.0, 11)])
    info, obs, P = c.transition(st, [0, 0, 0, 0], x)
    g = GOLD["E_depart_arrive"]
    assert (info.acc, info.rej, info.n_dep, info.M) == (g["acc"], g["rej"], g["n_dep"], 3)
    assert close(info.c_sat, g["c_sat"]) and close(info.reward, g["reward"])
    p2 = g["port2"]
    assert st.dwell[2] == p2["dwell"] and close(st.soc[2], p2["soc"]) and close(st.cap[2], p2["cap"])
    assert close(st.e_rem[2], p2["e_rem"]) and st.p_last[2] == 0.0
    assert list(st.dwell) == [4, 4, 7, 4]
    assert info.n_occ == 4


def test_first_free_port_and_reuse(oracle_lib):
    """Arrivals take the lowest-index free ports; a port freed this step is reusable."""
    o = oracle_lib
    spec = W.StationSpec(5, [-1], [1000.0], [1.0], [0] * 5, [22.0] * 5, [1.0] * 5)
    c = o.OracleClass(spec)
    st = o.EnvState(5)
    st.put_car(0, 0.5, 60.0, 3, 10.0)
    st.put_car(3, 0.5, 60.0, 1, 10.0)   # departs this step
    cars = [(41.0, 0.11, 0.71, 2), (42.0, 0.12, 0.72, 3), (43.0, 0.13, 0.73, 4)]
    info, _, _ = c.transition(st, [0] * 5, o.exo(3, 0.25, cars=cars))
    assert info.acc == 3 and info.rej == 0
    assert list(st.dwell) == [2, 2, 3, 4, 0]
    assert list(st.cap) == [60.0, 41.0, 42.0, 43.0, 0.0]


@pytest.mark.parametrize("d", [1, 2, 3, 7])
def test_dwell_counts_charging_steps(oracle_lib, d):
    """A car with dwell d charges in exactly d steps and leaves at the end of the d-th."""
    o = oracle_lib
    spec = W.StationSpec(1, [-1], [1000.0], [1.0], [0], [22.0], [1.0])
    c = o.OracleClass(spec)
    st = o.EnvState(1)
    st.put_car(0, 0.2, 80.0, d, 50.0)
    charged = 0
    for step in range(d + 2):
        info, _, P = c.transition(st, [10], o.exo(0, 0.25))
        charged += P[0] > 0
        if step == d - 1:
            assert info.n_dep == 1 and st.dwell[0] == 0
        else:
            assert info.n_dep == 0
    assert charged == d


def test_charge_closed_form(oracle_lib):
    """Full power with a non-binding tree: SoC rises by dt*pmax/C per step while SoC <= tau,
    then 1 - SoC shrinks by the factor 1 - dt*pmax/((1 - tau) C) per step (App. A.1-A.2)."""
    o = oracle_lib
    C_, dt, pmax, tau = 50.0, 1.0 / 12.0, 22.0, 0.8
    spec = W.StationSpec(1, [-1], [1000.0], [1.0], [0], [pmax], [1.0])
    c = o.OracleClass(spec)
    st = o.EnvState(1)
    st.put_car(0, 0.1, C_, 500, 100.0)
    lin = dt * pmax / C_
    geo = 1.0 - dt * pmax / ((1.0 - tau) * C_)
    n_lin = int(math.floor((tau - 0.1) / lin + 1e-12)) + 1   # steps started at SoC <= tau
    expect = []
    s = 0.1
    for n in range(60):
        if n < n_lin:
            s_next = 0.1 + (n + 1) * lin
        else:
            s_next = 1.0 - (1.0 - (0.1 + n_lin * lin)) * geo ** (n + 1 - n_lin)
        expect.append(s_next)
    got = []
    for n in range(60):
        c.transition(st, [10], o.exo(0, 0.25))
        got.append(st.soc[0])
    assert np.allclose(got, expect, rtol=0, atol=1e-12)


def test_day_boundary_resets(oracle_lib):
    o = oracle_lib
    spec = W.tiny_parity_station()
    c = o.OracleClass(spec)
    st = o.EnvState(16)
    st.put_car(3, 0.5, 60.0, 40, 20.0)
    st.t_day = 287
    info, obs, _ = c.transition(st, [10] * 16, o.exo(2, 0.25, cars=[(50, .2, .8, 5), (50, .2, .8, 5)]))
    assert info.done == 1 and st.t_day == 0 and info.acc == 2
    assert (st.dwell == 0).all() and (st.soc == 0).all()
    assert close(obs[:96], np.zeros(96)) and close(obs[96:], [0.0, 1.0, 0.25, 0.0])


def test_special_cases(oracle_lib):
    """All-zero actions give zero energy and reward -c_dt; huge limits never project."""
    o = oracle_lib
    spec = W.tiny_parity_station().replace(fixed_cost=0.3, price_sigma=0.0)
    c = o.OracleClass(spec)
    st = o.EnvState(16)
    for p in range(16):
        st.put_car(p, 0.3, 60.0, 9, 30.0)
    info, _, P = c.transition(st, [0] * 16, o.exo(0, 0.25))
    assert info.e_net == 0.0 and close(info.reward, -0.3)
    big = o.OracleClass(W.single_transformer(16, 1e6))
    req = np.linspace(0, 22, 16)
    assert np.array_equal(big.project(req), req)


def test_zero_rate_station_stays_empty(oracle_lib):
    o = oracle_lib
    spec = W.tiny_parity_station().replace(arrival_peak=0.0)
    c = o.OracleClass(spec)
    tp, _ = c.tables()
    assert (tp == 0xFFFFFFFF).all()
    bs = o.BatchState([c], np.zeros(8, np.int32))
    out = o.rollout(bs, 7, 600, want_info=True)
    assert out["info"]["M"].sum() == 0 and (bs.dwell == 0).all()
    assert np.all(out["reward"] == 0.0)
