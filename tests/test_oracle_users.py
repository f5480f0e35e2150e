"""Oracle pins for charge-sensitive users (App. A.1 "User Profiles", App. A.2
"Departure of Cars", App. A.3 c_satisfaction,1).

* hand-worked departures: a charge-sensitive user leaves at the end of the step
  in which the energy still wanted reaches zero -- early (c_satisfaction,1 =
  -beta x hours left) or late, past its planned departure (c_satisfaction,1 =
  hours overstayed) -- while a time-sensitive user beside it leaves on time;
* the model with (practically) no charge-sensitive users equals the base model
  step for step;
* the drawn share of charge-sensitive users is binomial with the given share;
* observations: the user flags, negative time left while overstaying, and the
  occupancy count include overstaying users.

Expected numbers are closed forms worked by hand, not oracle outputs.
"""
import math

import numpy as np
import pytest

import workloads as W

TOL = 1e-12
DT = 5.0 / 60.0


def close(a, b, tol=TOL):
    return np.allclose(np.asarray(a, float), np.asarray(b, float), rtol=tol, atol=tol)


def flat(n, **kw):
    base = dict(price_sigma=0.0, p_sell=0.45, p_sell_grid=0.25, arrival_peak=0.0,
                port_pmax_kw=[22.0] * n, port_eta=[1.0] * n, charge_sensitive_share=0.5,
                alpha_sat1=0.2, beta_sat1=0.5)
    base.update(kw)
    return W.StationSpec(n, [-1], [150.0], [1.0], [0] * n, **base)


def test_leaves_early_when_charged(oracle_lib):
    """5 kWh wanted at 22 kW: 22/12 kWh per step, charged during step 3 (e_rem
    5 - 3 * 22/12 = -0.5); 10 - 3 = 7 steps of its planned stay are left:
    c_satisfaction,1 = -beta * 7/12 h."""
    o = oracle_lib
    c = o.OracleClass(flat(1))
    st = c.new_state()
    st.put_car(0, 0.6, 50.0, 10, 5.0, user=1)
    for step in range(3):
        info, obs, P = c.transition(st, [10], o.exo(0, 0.25))
        assert close(P, [22.0])
        if step < 2:
            assert info.n_dep == 0 and st.user[0] == 1 and st.dwell[0] == 9 - step
    assert info.n_dep == 1 and st.user[0] == 0 and st.dwell[0] == 0 and st.cap[0] == 0.0
    assert close(info.c_sat1, -0.5 * 7.0 / 12.0)
    e = 22.0 / 12.0
    assert close(info.reward, 0.45 * e - 0.25 * e - 0.2 * (-0.5 * 7.0 / 12.0))


def test_overstays_until_charged(oracle_lib):
    """2 kWh wanted at level 1 (2.2 kW, 2.2/12 kWh per step): charged during the
    11th step (2 - 11 * 2.2/12 < 0 < 2 - 10 * 2.2/12); planned stay 2 steps, so
    it leaves 9 steps late: c_satisfaction,1 = 9/12 h.  The time-sensitive user
    beside it (same stay) leaves after step 2 with 2 - 2 * 2.2/12 kWh missing."""
    o = oracle_lib
    c = o.OracleClass(flat(2, alpha_sat=0.3))
    st = c.new_state()
    st.put_car(0, 0.5, 40.0, 2, 2.0, user=1)
    st.put_car(1, 0.5, 40.0, 2, 2.0, user=0)
    e = 2.2 / 12.0
    for step in range(11):
        info, obs, _ = c.transition(st, [1, 1], o.exo(0, 0.25))
        if step == 1:
            assert info.n_dep == 1 and st.dwell[1] == 0 and st.user[1] == 0
            assert close(info.c_sat, 2.0 - 2 * e)
        if step < 10:
            assert st.user[0] == 1 and st.dwell[0] == 1 - step
            assert info.c_sat1 == 0.0
            assert obs[0] == 1.0 and close(obs[3 * 2], (1 - step) / 288.0)   # occupied, time left
            assert obs[6 * 2 + 3] == (1.0 if step == 0 else 0.5)            # occupied share
            assert obs[6 * 2 + 4] == 1.0 and obs[6 * 2 + 5] == 0.0          # user flags
    assert info.n_dep == 1 and st.user[0] == 0 and st.dwell[0] == 0
    assert close(info.c_sat1, 9.0 / 12.0)
    assert close(info.reward, 0.45 * e - 0.25 * e - 0.2 * 9.0 / 12.0)


def test_arrivals_take_their_user_type(oracle_lib):
    o = oracle_lib
    c = o.OracleClass(flat(3))
    st = c.new_state()
    info, obs, _ = c.transition(st, [0, 0, 0], o.exo(2, 0.25, cars=[(50, .2, .8, 5, 1), (50, .2, .8, 5, 0)]))
    assert list(st.user) == [1, 0, 0] and list(st.dwell) == [5, 5, 0]
    assert list(obs[6 * 3 + 4:6 * 3 + 7]) == [1.0, 0.0, 0.0]


def test_share_of_charge_sensitive_users(oracle_lib):
    """The user type of car j of step g is Philox (env, g, j, USER) word 0 <= a
    threshold with (T + 1) / 2^32 = share: binomial counts."""
    o = oracle_lib
    for share in (0.3, 0.85):
        spec = flat(4, charge_sensitive_share=share, arrival_peak=3.0)
        c = o.OracleClass(spec)
        n = k = 0
        for env in range(30):
            for g in range(288):
                x = c.draw_exo(5, env, g, g)
                n += x.M
                k += sum(x.car_user[j] for j in range(x.M))
        assert n > 3000
        assert abs(k / n - share) < 5 * math.sqrt(share * (1 - share) / n)
    c = o.OracleClass(flat(4, charge_sensitive_share=1.0, arrival_peak=3.0))
    assert all(c.draw_exo(1, 0, g, g).car_user[j] == 1 for g in range(100) for j in range(c.draw_exo(1, 0, g, g).M))


@pytest.mark.parametrize("spec", [W.scale_station(), W.two_charger_types()], ids=["split16", "two_types"])
def test_no_charge_sensitive_users_is_the_base_model(oracle_lib, spec):
    """A share so small that no user is drawn charge-sensitive (threshold 0: only
    the word 0 would qualify) reproduces the base model's rewards, actions,
    flags and observations (plus an all-zero user block)."""
    o = oracle_lib
    busy = spec.replace(arrival_peak=2.0, alpha_sat=0.2)
    a = o.OracleClass(busy)
    b = o.OracleClass(busy.replace(charge_sensitive_share=1e-12, alpha_sat1=1.0, beta_sat1=0.5))
    ec = np.zeros(6, np.int32)
    ra = o.rollout(o.BatchState([a], ec), 7, 300)
    rb = o.rollout(o.BatchState([b], ec), 7, 300)
    N = spec.n_ports
    assert np.array_equal(ra["reward"], rb["reward"]) and np.array_equal(ra["act"], rb["act"])
    assert np.array_equal(ra["done"], rb["done"])
    ob = rb["obs"].reshape(300, 6, 7 * N + 4)
    assert np.array_equal(ra["obs"].reshape(300, 6, 6 * N + 4), ob[:, :, :6 * N + 4])
    assert not ob[:, :, 6 * N + 4:].any()


def test_rollout_invariants_with_users(oracle_lib):
    """A busy day and a half with 60 % charge-sensitive users: occupancy is
    conserved, time-sensitive users never hold negative time, only charged
    charge-sensitive users leave before their time, and the penalty terms add up
    to the reward."""
    o = oracle_lib
    spec = W.scale_station().replace(charge_sensitive_share=0.6, alpha_sat1=0.3, beta_sat1=0.4, alpha_sat=0.2,
                                     alpha_declined=0.1, arrival_peak=2.0)
    c = o.OracleClass(spec)
    st = c.new_state()
    n_cs_dep = n_late = 0
    for g in range(432):
        k = c.draw_actions(o.ACT_RANDOM, 6, 1, g)
        x = c.draw_exo(6, 1, g, st.t_day)
        occ0 = (st.dwell > 0) | (st.user == 1)
        user0, d0, e0 = st.user.copy(), st.dwell.copy(), st.e_rem.copy()
        info, obs, P = c.transition(st, k, x)
        occ1 = (st.dwell > 0) | (st.user == 1)
        assert np.all(st.dwell[st.user == 0] >= 0)
        if not info.done:
            assert occ1.sum() == occ0.sum() - info.n_dep + info.acc
            e = spec.dt_hours * P
            left = occ0 & ~occ1 | (occ0 & (st.dwell != d0 - 1))      # ports whose car left this step
            cs_left = left & (user0 == 1)
            assert np.all(e0[cs_left] - e[cs_left] <= 1e-12)           # they were charged
            n_cs_dep += int(cs_left.sum())
            n_late += int((cs_left & (d0 - 1 < 0)).sum())
        profit = info.profit
        assert close(info.reward, profit - 0.2 * info.c_sat - 0.1 * info.rej - 0.3 * info.c_sat1, 1e-9)
        assert obs[6 * 16 + 3] == occ1.sum() / 16.0
    assert n_cs_dep > 50 and n_late > 5
