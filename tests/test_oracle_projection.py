"""Oracle pins for the architecture projection of Eq. (ArchConst).

Brute force over every action vector of tiny stations (n <= 3 ports, trees of
depth <= 2) checks properties that fix the rescaling rule without re-stating
it: feasibility, identity when feasible, equal scaling of leaves that share the
same ancestors, no scaling without a binding constraint above the leaf, and
monotonicity in the actions.  The one-node case is compared with textbook
proportional scaling.
"""
import itertools

import numpy as np
import pytest

import workloads as W

REL = 1e-12

# (name, node_parent, node_limit, port_parent)
TREES = [
    ("flat2", [-1], [30.0], [0, 0]),
    ("flat3", [-1], [40.0], [0, 0, 0]),
    ("split2", [-1, 0], [25.0, 30.0], [1, 1]),
    ("split_mix", [-1, 0], [35.0, 20.0], [0, 1, 1]),
    ("two_splitters", [-1, 0, 0], [30.0, 25.0, 12.0], [1, 1, 2]),
    ("deep_chain", [-1, 0], [50.0, 18.0], [1, 0, 0]),
]


def leaves(node, node_parent, port_parent):
    out = []
    for i, p in enumerate(port_parent):
        a = p
        while a >= 0:
            if a == node:
                out.append(i)
                break
            a = node_parent[a]
    return out


def ancestors(i, node_parent, port_parent):
    s = []
    a = port_parent[i]
    while a >= 0:
        s.append(a)
        a = node_parent[a]
    return tuple(sorted(s))


@pytest.mark.parametrize("name,node_parent,node_limit,port_parent", TREES)
def test_projection_bruteforce(oracle_lib, name, node_parent, node_limit, port_parent):
    o = oracle_lib
    n = len(port_parent)
    spec = W.StationSpec(n, node_parent, node_limit, [1.0] * len(node_parent), port_parent,
                         [22.0] * n, [1.0] * n)
    c = o.OracleClass(spec)
    groups = {}
    for i in range(n):
        groups.setdefault(ancestors(i, node_parent, port_parent), []).append(i)
    node_leaves = [leaves(h, node_parent, port_parent) for h in range(len(node_parent))]
    dwell = np.full(n, 5, np.int32)
    soc = np.full(n, 0.5)
    cap = np.full(n, 60.0)
    results = {}
    for k in itertools.product(range(11), repeat=n):
        req = np.array(k, float) / 10.0 * 22.0
        P = c.apply_actions(dwell, soc, cap, k)
        results[k] = P
        # feasibility of every node
        for h, lv in enumerate(node_leaves):
            assert P[lv].sum() <= node_limit[h] * (1 + REL)
        feasible = all(req[lv].sum() <= node_limit[h] for h, lv in enumerate(node_leaves))
        if feasible:
            assert np.array_equal(P, req)
        assert np.all(P <= req * (1 + REL)) and np.all(P >= 0)
        # leaves with the same ancestor set are scaled by the same factor
        for grp in groups.values():
            r = [P[i] / req[i] for i in grp if req[i] > 0]
            assert np.allclose(r, r[0] if r else 0, rtol=1e-12)
        # a scaled leaf has a binding constraint on its path
        for i in range(n):
            if req[i] > 0 and P[i] < req[i] * (1 - 1e-12):
                anc = ancestors(i, node_parent, port_parent)
                assert any(abs(P[node_leaves[h]].sum() - node_limit[h]) <= 1e-9 * node_limit[h]
                           for h in anc)
    # monotone: raising one port's level never lowers its power nor raises another's
    for k, P in results.items():
        for i in range(n):
            if k[i] < 10:
                k2 = list(k)
                k2[i] += 1
                P2 = results[tuple(k2)]
                assert P2[i] >= P[i] * (1 - 1e-12)
                others = [j for j in range(n) if j != i]
                assert np.all(P2[others] <= P[others] * (1 + 1e-12) + 1e-12)


def test_single_node_is_textbook_scaling(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(0)
    c = o.OracleClass(W.single_transformer(16, 150.0))
    for _ in range(200):
        req = rng.uniform(0, 22, 16) * (rng.uniform() < 0.8)
        P = c.project(req)
        s = req.sum()
        expect = req * (150.0 / s) if s > 150.0 else req
        assert np.allclose(P, expect, rtol=1e-13, atol=0)


def test_deep_trees_feasible(oracle_lib):
    """Every node of the 15 mixture classes is within its limit after projection."""
    o = oracle_lib
    rng = np.random.default_rng(1)
    for spec in W.mixture_classes():
        c = o.OracleClass(spec)
        node_leaves = [leaves(h, spec.node_parent, spec.port_parent) for h in range(spec.n_nodes)]
        for _ in range(20):
            req = rng.integers(0, 11, spec.n_ports) / 10.0 * 22.0
            P = c.project(req)
            for h, lv in enumerate(node_leaves):
                assert P[lv].sum() <= spec.node_limit_kw[h] * (1 + 1e-12)
