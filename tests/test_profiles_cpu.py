"""Time-of-day profiles (per-step Poisson arrival means and base prices, Sec. 3
"Exogenous State Space", Table 1): oracle pins against scipy and closed forms,
and the library's host-built tables against the oracle's."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    return cx


def test_poisson_table_follows_given_rates(oracle_lib):
    """T[t][k] = ceil(2^32 F(k; lambda_t)) - 1 for the given per-step means."""
    spec = W.profile_station()
    tp, _ = oracle_lib.OracleClass(spec).tables()
    for t in range(spec.steps_per_episode):
        lam = spec.arrival_rate[t]
        cdf = stats.poisson.cdf(np.arange(24), lam)
        approx = (tp[t].astype(np.float64) + 1) / 2**32
        assert np.all(np.abs(approx - cdf) <= 2.0**-32 + 1e-13), t


def test_price_table_sets_buy_price_and_observation(oracle_lib):
    """With the price noise switched off, p_buy at step t is the table entry, and
    the observation's base-price feature is the table entry of the current step."""
    o = oracle_lib
    spec = W.profile_station().replace(price_sigma=0.0)
    c = o.OracleClass(spec)
    for t in (0, 30, 100, 210, 250, 287):
        assert c.draw_exo(3, 1, t, t).p_buy == spec.price_table[t]
        st = o.EnvState(spec.n_ports)
        st.t_day = t
        assert c.observe(st)[6 * spec.n_ports + 2] == spec.price_table[t]


def test_zero_rate_steps_have_no_arrivals(oracle_lib):
    """lambda_t = 0 gives the all-ones threshold row (no arrivals); arrivals only
    at the steps with a positive mean, and their daily mean is the sum of means."""
    o = oracle_lib
    rate = np.zeros(288)
    rate[[10, 100, 200]] = [0.5, 2.0, 1.0]
    spec = W.tiny_parity_station().replace(arrival_rate=rate)
    c = o.OracleClass(spec)
    tp, _ = c.tables()
    assert np.all(tp[rate == 0] == 0xFFFFFFFF)
    M = np.array([[c.draw_exo(7, e, t, t).M for t in range(288)] for e in range(300)])
    assert not M[:, rate == 0].any()
    for t in (10, 100, 200):
        assert abs(M[:, t].mean() - rate[t]) < 5 * math.sqrt(rate[t] / 300)


def test_default_profiles_unchanged(oracle_lib):
    """Profiles equal to the default curves reproduce the default tables exactly."""
    base = W.tiny_parity_station()
    S = base.steps_per_episode
    t = np.arange(S)
    rate = 0.5 * base.arrival_peak * (1 - np.cos(2 * np.pi * t / S))
    price = base.price_base + base.price_amp * np.sin(2 * np.pi * t / S)
    a = oracle_lib.OracleClass(base).tables()[0]
    b = oracle_lib.OracleClass(base.replace(arrival_rate=rate, price_table=price)).tables()[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("spec", [W.profile_station(),
                                  W.fanout4_tree(64, 2).replace(arrival_rate=W.commuter_arrivals() * 4),
                                  W.tiny_parity_station().replace(price_table=W.time_of_use_prices())])
def test_library_tables_equal_oracle(cxm, oracle_lib, spec):
    tp, td = cxm.build_tables(spec)
    otp, otd = oracle_lib.OracleClass(spec).tables()
    assert np.array_equal(tp, otp)
    assert np.array_equal(td[1:], otd[1:])


def test_profile_validation(cxm):
    bad = W.tiny_parity_station().replace(arrival_rate=np.full(288, 9.0))
    with pytest.raises(cxm.CxError):
        cxm.build_tables(bad)
    nan = W.tiny_parity_station().replace(price_table=np.full(288, np.nan))
    with pytest.raises(cxm.CxError):
        cxm.build_tables(nan)
    with pytest.raises(ValueError):
        cxm.build_tables(W.tiny_parity_station().replace(price_table=np.zeros(10)))
