"""Random capacity trees (workloads.random_station: 1-4 levels, 1-4 children per
node, ports under leaves and inner nodes, random limits, efficiencies, port
maxima, level counts): the library either compiles them or refuses the ones
whose aligned layout would exceed 256 slots, never anything else; the integer
sampling tables of the accepted ones equal the oracle's; and the oracle runs
them (its projection keeps every node within its limit)."""
import numpy as np
import pytest

import workloads as W

SEEDS = range(60)


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    cx.lib()
    return cx


def accepted(cxm, seeds=SEEDS, max_ports=40):
    out = []
    for s in seeds:
        spec = W.random_station(s, max_ports=max_ports)
        try:
            cxm.compile_layout(spec)
        except cxm.CxError as e:
            assert "256 slots" in str(e), (s, str(e))
            continue
        out.append(spec)
    return out


def test_random_trees_compile_or_are_refused_for_size(cxm):
    specs = accepted(cxm)
    assert len(specs) >= 50
    assert {len(s.node_parent) for s in specs} >= {1}
    assert max(s.n_ports for s in specs) == 40 and min(s.n_ports for s in specs) <= 3


def test_random_trees_tables_equal_oracle(cxm, oracle_lib):
    for spec in accepted(cxm, range(12)):
        tp, td = cxm.build_tables(spec)
        otp, otd = oracle_lib.OracleClass(spec).tables()
        assert np.array_equal(tp, otp), spec.name
        assert np.array_equal(td[1:], otd[1:]), spec.name


def test_random_trees_oracle_respects_limits(cxm, oracle_lib):
    """Max levels on busy stations: after every projection each node's net
    power is within its limit (the oracle's P out of the transition)."""
    o = oracle_lib
    for spec in accepted(cxm, range(8)):
        c = o.OracleClass(spec.replace(arrival_peak=4.0))
        st = c.new_state()
        for g in range(40):
            k = c.draw_actions(o.ACT_MAX, 0, 0, g)
            x = c.draw_exo(0, 0, g, st.t_day)
            _, _, P = c.transition(st, k, x)
            for h, lim in enumerate(spec.node_limit_kw):
                under = [i for i in range(spec.n_ports) if h in ancestors(spec, spec.port_parent[i])]
                assert sum(P[i] for i in under) <= lim * (1 + 1e-9) + 1e-9, (spec.name, h)


def ancestors(spec, h):
    out = []
    while h >= 0:
        out.append(h)
        h = spec.node_parent[h]
    return out
