"""Oracle pins for exploring starts (Supp. B.1: at every reset a random day of
the price data is drawn and its prices are used for the episode; the agent
observes the day and whether it is a weekday).

* the day of an episode is uniform over the price days (chi-square), fixed for
  the whole episode and a function of (env, first step) alone;
* with the noise off, the buying price of every step is the drawn day's row,
  and the observation shows that row's next price, day / n_days and the weekend
  flag (day mod 7 >= 5);
* one price day equal to the per-step price table gives the table model's
  records exactly (plus the two day features).
"""
import numpy as np
import pytest
from scipy import stats

import workloads as W


def days_spec(n_days=10, **kw):
    s = W.tiny_parity_station().replace(price_days=W.price_day_table(n_days), **kw)
    return s


def test_days_uniform_and_per_episode(oracle_lib):
    o = oracle_lib
    spec = days_spec(10)
    c = o.OracleClass(spec)
    draws = [c.episode_day(3, env, 288 * k) for env in range(200) for k in range(10)]
    cnt = np.bincount(draws, minlength=10)
    assert cnt.sum() == 2000 and stats.chisquare(cnt).pvalue > 1e-4
    # constant within an episode: every step of the episode starting at g0 reports that day
    for env, g0 in ((0, 0), (5, 288), (17, 1000)):
        d0 = c.episode_day(3, env, g0)
        for t in (0, 1, 150, 287):
            x = c.draw_exo(3, env, g0 + t, t)
            assert x.day == d0
        assert c.draw_exo(3, env, g0 + 287, 287).day_next == c.episode_day(3, env, g0 + 288)
        assert c.draw_exo(3, env, g0 + 5, 5).day_next == d0
    assert c.episode_day(3, 4, 0) == o.OracleClass(spec).episode_day(3, 4, 0)      # deterministic
    assert o.OracleClass(W.tiny_parity_station()).episode_day(3, 4, 0) == -1    # no days: none drawn


def test_prices_and_observation_follow_the_day(oracle_lib):
    o = oracle_lib
    spec = days_spec(10, price_sigma=0.0)
    table = spec.price_days
    c = o.OracleClass(spec)
    seed, env = 9, 3
    st = c.new_state(seed, env, 0)
    N = spec.n_ports
    seen = set()
    for g in range(3 * 288):
        x = c.draw_exo(seed, env, g, st.t_day)
        d = c.episode_day(seed, env, g - st.t_day)
        assert x.day == d == st.day and x.p_buy == table[d, st.t_day]
        seen.add(d)
        k = c.draw_actions(o.ACT_RANDOM, seed, env, g)
        info, obs, _ = c.transition(st, k, x)
        dn = st.day
        assert obs[6 * N + 2] == table[dn, st.t_day]
        assert obs[6 * N + 4] == dn / 10 and obs[6 * N + 5] == (1.0 if dn % 7 >= 5 else 0.0)
        if info.done:
            assert dn == c.episode_day(seed, env, g + 1)
    assert len(seen) >= 2


def test_one_day_is_the_price_table(oracle_lib):
    o = oracle_lib
    prices = W.time_of_use_prices()
    a = W.scale_station().replace(price_table=prices, arrival_peak=1.0, alpha_sat=0.1)
    b = a.replace(price_table=None, price_days=prices[None, :])
    ec = np.zeros(5, np.int32)
    ra = o.rollout(o.BatchState([o.OracleClass(a)], ec), 2, 600)
    rb = o.rollout(o.BatchState([o.OracleClass(b)], ec), 2, 600)
    assert np.array_equal(ra["reward"], rb["reward"]) and np.array_equal(ra["act"], rb["act"])
    N = a.n_ports
    oa, ob = ra["obs"].reshape(600, 5, -1), rb["obs"].reshape(600, 5, -1)
    assert ob.shape[2] == 6 * N + 6
    assert np.array_equal(oa, ob[:, :, :6 * N + 4])
    assert (ob[:, :, 6 * N + 4:] == 0).all()                                   # day 0 of 1, a weekday


def test_weekend_flag_every_day(oracle_lib):
    """Every day 0..9 observed at an episode start: day / 10 and the weekend flag
    (days 5, 6 of each week are weekend days)."""
    o = oracle_lib
    spec = days_spec(10)
    c = o.OracleClass(spec)
    N = spec.n_ports
    found = {}
    env = 0
    while len(found) < 10:
        d = c.episode_day(1, env, 0)
        found.setdefault(d, env)
        env += 1
    for d, env in sorted(found.items()):
        obs = c.observe(c.new_state(1, env, 0))
        assert obs[6 * N + 4] == d / 10
        assert obs[6 * N + 5] == (1.0 if d in (5, 6) else 0.0), d
        assert obs[6 * N + 2] == spec.price_days[d, 0]
