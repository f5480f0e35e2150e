"""CPU checks of the HIP library's host side: it loads, exports every symbol the
headers declare, validates specs, compiles capacity trees into the aligned slot
layout, and builds integer sampling tables identical to the oracle's (the hard
gate for integer bit-exactness).  No kernel is launched."""
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    cx.lib()
    return cx


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)          # drop comments
            names |= set(re.findall(r"(?:cx_status|void|char\s*\*)\s+(cx_[a-z_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol(cxm):
    names = declared_symbols()
    assert len(names) >= 25
    L = cxm.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing
    assert set(cxm.EXPORTS) >= names


SPECS = [W.tiny_parity_station(), W.scale_station(), W.policy_station(), W.two_charger_types(),
         W.tiny_parity_station().replace(arrival_peak=0.0, dwell_max=1),
         W.fanout4_tree(32, 2).replace(steps_per_episode=96, dwell_max=300, dwell_mu=math.log(12.0)),
         W.fanout4_tree(128, 3).replace(arrival_peak=8.0)] + W.mixture_classes() + W.v2g_mixture() + \
        [W.user_station(), W.exo_station()]


@pytest.mark.parametrize("spec", SPECS, ids=[s.name or str(i) for i, s in enumerate(SPECS)])
def test_tables_equal_oracle(cxm, oracle_lib, spec):
    tp, td = cxm.build_tables(spec)
    otp, otd = oracle_lib.OracleClass(spec).tables()
    assert np.array_equal(tp, otp)
    assert np.array_equal(td[1:], otd[1:])


def leaves_of(spec, h):
    out = []
    for i, p in enumerate(spec.port_parent):
        a = p
        while a >= 0:
            if a == h:
                out.append(i)
                break
            a = spec.node_parent[a]
    return out


@pytest.mark.parametrize("spec", SPECS[:4] + W.mixture_classes() + W.v2g_mixture(), ids=lambda s: s.name)
def test_layout_is_aligned_and_order_preserving(cxm, spec):
    lay = cxm.compile_layout(spec)
    S, D = lay["slots"], lay["levels"]
    port = lay["slot_port"]
    assert S >= spec.n_ports and S & (S - 1) == 0
    used = port[port >= 0]
    assert np.array_equal(used, np.arange(spec.n_ports))          # port order = slot order
    depth = [0] * spec.n_nodes
    for h in range(1, spec.n_nodes):
        depth[h] = depth[spec.node_parent[h]] + 1
    assert D == max(depth) + 1
    slot_of = {int(p): s for s, p in enumerate(port) if p >= 0}
    for h in range(spec.n_nodes):
        lvl = D - 1 - depth[h]
        slots = [slot_of[i] for i in leaves_of(spec, h)]
        lb = (lay["slot_lb"][slots] >> (8 * lvl)) & 0xFF
        assert len(set(lb.tolist())) == 1
        if h > 0 and lb[0] & 0x80:                                 # dense level: node code, exact cover
            cover = np.flatnonzero(((lay["slot_lb"] >> (8 * lvl)) & 0xFF) == lb[0])
            assert sorted(cover.tolist()) == sorted(slots)
            assert np.allclose(lay["slot_cap"][lvl, slots], spec.node_limit_kw[h] * spec.node_eta[h])
            continue
        B = 1 << int(lb[0])
        base = min(slots) // B * B
        assert max(slots) < base + B                               # one aligned block holds the subtree
        assert np.allclose(lay["slot_cap"][lvl, base:base + B], spec.node_limit_kw[h] * spec.node_eta[h])


def test_uneven_tree_layouts(cxm):
    """A tree whose aligned layout would pad takes the dense layout when each
    level below the root has at most 4 nodes; otherwise it is padded."""
    lay = cxm.compile_layout(W.two_charger_types())                 # 10 DC + 6 AC ports: dense, 16 slots
    assert lay["slots"] == 16 and lay["levels"] == 2
    assert list(lay["slot_port"]) == list(range(16))
    lvl0 = lay["slot_lb"] & 0xFF
    assert list(lvl0) == [0x80] * 10 + [0x81] * 6
    assert list(lay["slot_cap"][0]) == [800.0] * 10 + [50.0] * 6
    # five splitters of 3 ports: more than 4 nodes on a level, so the aligned layout pads (4 per block)
    five = W.splitter_tree(5, 3, 30.0, 100.0)
    lay = cxm.compile_layout(five)
    assert lay["slots"] == 32 and not (lay["slot_lb"] & 0x80).any()
    assert list(lay["slot_port"][:8]) == [0, 1, 2, -1, 3, 4, 5, -1]
    # 4 + 3 ports: the aligned layout does not pad (8 slots), so it stays aligned
    lay = cxm.compile_layout(W.StationSpec(7, [-1, 0, 0], [50.0, 30.0, 30.0], [1.0] * 3, [1] * 4 + [2] * 3,
                                           [22.0] * 7, [1.0] * 7))
    assert lay["slots"] == 8 and not (lay["slot_lb"] & 0x80).any()
    # 5 + 2 ports: aligned would take 16 slots; dense takes 8, the padding slot covered by no node
    lay = cxm.compile_layout(W.StationSpec(7, [-1, 0, 0], [50.0, 30.0, 30.0], [1.0] * 3, [1] * 5 + [2] * 2,
                                           [22.0] * 7, [1.0] * 7))
    assert lay["slots"] == 8 and list(lay["slot_lb"] & 0xFF) == [0x80] * 5 + [0x81] * 2 + [0]


BAD = [
    ("n_ports", dict(n_ports=0, port_parent=[], port_pmax_kw=[], port_eta=[])),
    ("node_parent", dict(node_parent=[0])),
    ("limits", dict(node_limit_kw=[-1.0])),
    ("tau", dict(tau=1.0)),
    ("eta", dict(port_eta=[0.0] * 16)),
    ("dfs", None),
    ("depth", None),
    ("v2g_flag", dict(v2g=2)),
    ("pdis", dict(v2g=1, port_pdis_kw=[0.0] * 16)),
    ("v2g_levels", dict(v2g=1, n_levels=200)),
    ("battery_rate", dict(battery_kwh=50.0, battery_kw=0.0)),
    ("battery_tau", dict(battery_kwh=50.0, battery_kw=10.0, battery_tau=1.0)),
    ("battery_soc0", dict(battery_kwh=50.0, battery_kw=10.0, battery_soc0=1.5)),
    ("battery_kwh", dict(battery_kwh=float("nan"))),
    ("cs_share", dict(charge_sensitive_share=1.5)),
    ("cs_alpha", dict(charge_sensitive_share=0.5, alpha_sat1=float("inf"))),
    ("cs_long_episode", dict(charge_sensitive_share=0.5, steps_per_episode=40000)),
    ("price_days_nan", dict(price_days=np.full((3, 288), np.nan))),
    ("car_model_sum", dict(car_models=np.array([[0.5, 40.0, 7.0, 50.0], [0.4, 60.0, 11.0, 100.0]]))),
    ("car_model_rate", dict(car_models=np.array([[1.0, 40.0, 0.0, 50.0]]))),
    ("port_dc", dict(car_models=np.array([[1.0, 40.0, 7.0, 50.0]]), port_dc=[2] * 16)),
]


@pytest.mark.parametrize("what,kw", BAD)
def test_invalid_specs_rejected(cxm, what, kw):
    if what == "dfs":
        spec = W.StationSpec(4, [-1, 0, 0], [100, 50, 50], [1, 1, 1], [1, 2, 1, 2], [22.0] * 4, [1.0] * 4)
    elif what == "depth":
        spec = W.StationSpec(1, [-1, 0, 1, 2, 3], [9.0] * 5, [1.0] * 5, [4], [22.0], [1.0])
    else:
        spec = W.tiny_parity_station().replace(**kw)
    with pytest.raises(cxm.CxError) as ei:
        cxm.compile_layout(spec)
    assert ei.value.status == -1 and str(ei.value)


def test_noalloc_scratch_size_matches_header(cxm):
    txt = open(os.path.join(ROOT, "include", "cx.h")).read()
    m = re.search(r"#define CX_NOALLOC_SCRATCH_BYTES (\d+)", txt)
    assert m and int(m.group(1)) == cxm.NOALLOC_SCRATCH_BYTES


def test_noalloc_refuses_without_context(cxm):
    assert cxm.lib().cx_rollout_policy_noalloc(None, 4, cxm.OUT_FULL, None) == -1
