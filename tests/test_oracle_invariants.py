"""Oracle pins: invariants of whole rollouts (App. A.2-A.3, Supp. B.1).

  * every capacity node within its limit, every SoC within [0, 1];
  * delivered energy = summed SoC gains x battery capacity; grid energy = sum e / eta;
  * occupancy conserved: occ_t = occ_{t-1} - departures + accepted;
  * accepted + rejected = arrivals; done exactly every 288 steps;
  * the batched rollout equals the one-env transition loop, and envs are
    independent of one another and of the thread split.
"""
import numpy as np
import pytest

import workloads as W


def node_leaves(spec):
    out = []
    for h in range(spec.n_nodes):
        lv = []
        for i, p in enumerate(spec.port_parent):
            a = p
            while a >= 0:
                if a == h:
                    lv.append(i)
                    break
                a = spec.node_parent[a]
        out.append(lv)
    return out


@pytest.mark.parametrize("spec", [W.scale_station().replace(port_eta=[0.9] * 8 + [0.95] * 8),
                                  W.fanout4_tree(32, 3), W.two_charger_types()],
                         ids=["split16_eta", "fan32d3", "two_types"])
def test_rollout_invariants(oracle_lib, spec):
    o = oracle_lib
    c = o.OracleClass(spec.replace(arrival_peak=spec.arrival_peak * 3))   # busier station
    lv = node_leaves(spec)
    caps = [spec.node_limit_kw[h] * spec.node_eta[h] for h in range(spec.n_nodes)]
    st = o.EnvState(spec.n_ports)
    n_done = 0
    for g in range(2 * 288 + 17):
        k = c.draw_actions(o.ACT_RANDOM, 8, 3, g)
        x = c.draw_exo(8, 3, g, st.t_day)
        before = (st.dwell.copy(), st.soc.copy(), st.cap.copy(), st.t_day)
        info, obs, P = c.transition(st, k, x)
        d0, s0, c0, t0 = before
        occ0 = d0 > 0
        for h in range(spec.n_nodes):
            assert P[lv[h]].sum() <= caps[h] * (1 + 1e-12)
        assert np.all(P[~occ0] == 0)
        e = spec.dt_hours * P
        assert np.isclose(info.e_net, e.sum(), rtol=1e-12, atol=1e-12)
        assert np.isclose(info.e_grid, (e / np.array(spec.port_eta)).sum(), rtol=1e-12, atol=1e-12)
        # SoC gain x capacity equals delivered energy for cars that stay
        stay = occ0 & (st.dwell > 0) & (st.dwell == d0 - 1)
        assert np.allclose((st.soc[stay] - s0[stay]) * c0[stay], e[stay], rtol=1e-9, atol=1e-12)
        assert np.all((st.soc >= 0) & (st.soc <= 1))
        assert info.acc + info.rej == info.M
        if info.done:
            n_done += 1
            assert t0 == 287 and st.t_day == 0 and info.n_occ == 0
        else:
            assert info.n_occ == occ0.sum() - info.n_dep + info.acc
            assert st.t_day == t0 + 1
    assert n_done == 2


def test_energy_balance_over_car_lifetimes(oracle_lib):
    """Summed E_net over a day = summed (final SoC - initial SoC) x C over all cars."""
    o = oracle_lib
    spec = W.tiny_parity_station().replace(arrival_peak=0.6)
    c = o.OracleClass(spec)
    st = o.EnvState(16)
    total_e, gained = 0.0, 0.0
    for g in range(287):
        k = c.draw_actions(o.ACT_RANDOM, 21, 0, g)
        x = c.draw_exo(21, 0, g, st.t_day)
        d0, s0, c0 = st.dwell.copy(), st.soc.copy(), st.cap.copy()
        info, _, P = c.transition(st, k, x)
        total_e += info.e_net
        occ0 = d0 > 0
        leaving = occ0 & (d0 == 1)
        # a departing car's last SoC is s0 + e/C (no clamp binds for these parameters)
        final = np.minimum(1.0, s0 + spec.dt_hours * P / np.where(occ0, c0, 1))
        gained += (final * c0)[leaving].sum()
        arrived = (st.dwell > 0) & ~(occ0 & ~leaving)
        gained -= (st.soc * st.cap)[arrived].sum()
    occ = st.dwell > 0
    gained += (st.soc * st.cap)[occ].sum()
    # each car adds (final SoC) x C when it leaves or at the end and subtracts SoC_0 x C on arrival
    assert np.isclose(total_e, gained, rtol=1e-10)


def test_batched_equals_single_env_loop(oracle_lib):
    o = oracle_lib
    classes = [o.OracleClass(W.fanout4_tree(8, 2)), o.OracleClass(W.scale_station())]
    env_class = np.array([1, 0, 1, 1, 0], np.int32)
    bs = o.BatchState(classes, env_class)
    out = o.rollout(bs, 77, 300, want_info=True, n_threads=3)
    for e, ci in enumerate(env_class):
        c = classes[ci]
        st = o.EnvState(c.n)
        po = int(bs.port_off[e])
        oo = int(bs.obs_off[e])
        for g in range(300):
            k = c.draw_actions(o.ACT_RANDOM, 77, e, g)
            x = c.draw_exo(77, e, g, st.t_day)
            info, obs, _ = c.transition(st, k, x)
            assert out["reward"][g, e] == info.reward
            assert np.array_equal(out["obs"][g, oo:oo + c.obs_dim], obs)
            assert np.array_equal(out["act"][g, po:po + c.n], k)
        assert np.array_equal(bs.dwell[po:po + c.n], st.dwell)
        assert np.array_equal(bs.soc[po:po + c.n], st.soc)
        assert bs.ret[e] == st.ret
    # thread split does not matter
    bs2 = o.BatchState(classes, env_class)
    out2 = o.rollout(bs2, 77, 300, n_threads=1)
    assert np.array_equal(out2["obs"], out["obs"]) and np.array_equal(bs2.ret, bs.ret)


def test_snapshot_resume_equals_uninterrupted(oracle_lib):
    o = oracle_lib
    cls = [o.OracleClass(W.scale_station())]
    a = o.BatchState(cls, np.zeros(6, np.int32))
    full = o.rollout(a, 5, 400)
    b = o.BatchState(cls, np.zeros(6, np.int32))
    first = o.rollout(b, 5, 150)
    second = o.rollout(b, 5, 250)
    assert np.array_equal(np.concatenate([first["obs"], second["obs"]]), full["obs"])
    assert np.array_equal(b.soc, a.soc) and b.g == a.g == 400 and b.t_day == a.t_day == 400 % 288
