"""Oracle pins for car models (App. A.1 "Car Profiles": a capacity and a maximum
rate per charger type, AC and DC, sampled from a car distribution; both curves
share tau).

* model frequencies follow the given probabilities (chi-square);
* hand-worked clips: the same car draws its AC rate at an AC port and its DC
  rate at a DC port, tapering above tau from that rate; the observation's
  r_hat / pmax uses it;
* one model whose rates equal the port maxima and whose capacity is fixed gives
  the base model's records exactly;
* over a busy rollout no port ever draws more than its car's curve allows.
"""
import numpy as np
import pytest
from scipy import stats

import workloads as W

TOL = 1e-12


def close(a, b, tol=TOL):
    return np.allclose(np.asarray(a, float), np.asarray(b, float), rtol=tol, atol=tol)


def two_type(models, **kw):
    base = dict(price_sigma=0.0, arrival_peak=0.0, car_models=np.asarray(models, float), port_dc=[0, 1])
    base.update(kw)
    return W.StationSpec(2, [-1], [500.0], [1.0], [0, 0], [11.5, 150.0], [1.0, 1.0], **base)


def test_model_frequencies(oracle_lib):
    o = oracle_lib
    spec = W.exo_station()
    c = o.OracleClass(spec)
    counts = np.zeros(4)
    n = 0
    for env in range(60):
        for g in range(288):
            x = c.draw_exo(2, env, g, g)
            for j in range(x.M):
                counts[x.car_model[j]] += 1
                assert x.car_cap[j] == spec.car_models[x.car_model[j], 1]
            n += x.M
    assert n > 3000
    assert stats.chisquare(counts, spec.car_models[:, 0] * n).pvalue > 1e-4


def test_ac_and_dc_rates(oracle_lib):
    """One car model (60 kWh, 7.4 kW AC, 50 kW DC); an AC port of 11.5 kW and a
    DC port of 150 kW.  Flat part: 7.4 and 50 kW.  At SoC 0.9 (tau 0.8): the
    taper (1 - 0.9) / 0.2 of the car's rate: 3.7 and 25 kW."""
    o = oracle_lib
    c = o.OracleClass(two_type([[1.0, 60.0, 7.4, 50.0]]))
    st = c.new_state()
    info, obs, P = c.transition(st, [0, 0], o.exo(2, 0.25, cars=[(60.0, 0.5, 0.9, 20, 0, 0), (60.0, 0.5, 0.9, 20, 0, 0)]))
    assert close(st.rbar, [7.4, 50.0]) and close(st.cap, [60.0, 60.0])
    assert close(obs[4 * 2:5 * 2], [7.4 / 11.5, 50.0 / 150.0])      # r_hat / pmax
    info, obs, P = c.transition(st, [10, 10], o.exo(0, 0.25))
    assert close(P, [7.4, 50.0])
    st.soc[:] = 0.9
    info, obs, P = c.transition(st, [10, 10], o.exo(0, 0.25))
    assert close(P, [3.7, 25.0])
    # a level below the car's rate is not clipped by it
    st.soc[:] = 0.5
    info, obs, P = c.transition(st, [2, 2], o.exo(0, 0.25))
    assert close(P, [2.3, 30.0])


def test_one_model_is_the_base_model(oracle_lib):
    """A single 60 kWh model whose AC and DC rates are the ports' maxima equals
    the base model with capacities fixed at 60 kWh."""
    o = oracle_lib
    base = W.two_charger_types().replace(cap_lo=60.0, cap_hi=60.0, arrival_peak=2.0, alpha_sat=0.2)
    cars = base.replace(car_models=np.array([[1.0, 60.0, 11.5, 150.0]]), port_dc=[1] * 10 + [0] * 6)
    ec = np.zeros(6, np.int32)
    ra = o.rollout(o.BatchState([o.OracleClass(base)], ec), 3, 400)
    rb = o.rollout(o.BatchState([o.OracleClass(cars)], ec), 3, 400)
    for k in ("reward", "act", "done", "obs"):
        assert np.array_equal(ra[k], rb[k]), k


def test_never_above_the_cars_curve(oracle_lib):
    o = oracle_lib
    spec = W.exo_station(arrival_rate=W.commuter_arrivals() * 3)
    c = o.OracleClass(spec)
    st = c.new_state(4, 1, 0)
    tau = spec.tau
    n_bind = 0
    for g in range(400):
        k = c.draw_actions(o.ACT_RANDOM, 4, 1, g)
        x = c.draw_exo(4, 1, g, st.t_day)
        occ = st.dwell > 0
        soc, rb = st.soc.copy(), st.rbar.copy()
        info, obs, P = c.transition(st, k, x)
        rhat = np.where(soc <= tau, rb, (1 - soc) * rb / (1 - tau))
        assert np.all(P[occ] <= rhat[occ] * (1 + 1e-12))
        assert np.all(rb[occ] > 0)
        n_bind += int(np.sum(np.isclose(P[occ], rhat[occ]) & (rhat[occ] < np.array(spec.port_pmax_kw)[occ])))
    assert n_bind > 50
