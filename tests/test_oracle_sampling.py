"""Oracle pins for the random parts: Philox, the integer sampling tables and the
statistics of every exogenous draw (App. A.1 exogenous state; Supp. B.1 Poisson
arrivals; Sec. 3 grid prices; discretised actions).

Independent references: published Philox known-answer vectors, rocRAND's own
Philox implementation (compiled from its source headers), scipy's Poisson and
lognormal distributions, and closed-form moments.
"""
import json
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers(oracle_lib):
    kat = json.load(open(os.path.join(HERE, "golden", "philox_kat.json")))["vectors"]
    for v in kat:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(oracle_lib.philox(ctr, key)) == out


ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct E : rocrand_device::philox4x32_10_engine { using philox4x32_10_engine::ten_rounds; };
int main() {
  E e; unsigned a, b, c, d, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
    uint4 r = e.ten_rounds(uint4{a, b, c, d}, uint2{k0, k1});
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available for the rocRAND cross-check")
def test_philox_matches_rocrand_headers(oracle_lib):
    """A second, independent Philox4x32-10 (rocRAND's header) agrees on random inputs."""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "x.cpp")
        exe = os.path.join(d, "x")
        open(src, "w").write(ROCRAND_SRC)
        subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-o", exe, src],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        rng = np.random.default_rng(42)
        inp = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
        inp[:8, 1] = np.arange(8)          # counters of the shapes the simulator uses
        txt = "\n".join(" ".join(str(int(v)) for v in row) for row in inp)
        res = subprocess.run([exe], input=txt.encode(), capture_output=True, check=True).stdout.decode()
        ref = np.array([[int(x) for x in ln.split()] for ln in res.strip().splitlines()], dtype=np.uint64)
    for row, r in zip(inp, ref):
        assert list(oracle_lib.philox(row[:4], row[4:])) == list(r)


def test_philox_bit_balance(oracle_lib):
    words = np.array([oracle_lib.philox((e, g, 0, 0), (1, 0)) for e in range(64) for g in range(64)],
                     dtype=np.uint64).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=0)
    n = words.size
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(n))


def test_poisson_table_matches_scipy(oracle_lib):
    """T[t][k] = ceil(2^32 F(k; lambda(t))) - 1 with lambda(t) = peak (1 - cos 2 pi t/S) / 2."""
    for spec in [W.tiny_parity_station(), W.fanout4_tree(128, 3)]:
        c = oracle_lib.OracleClass(spec)
        tp, _ = c.tables()
        S = spec.steps_per_episode
        for t in range(S):
            lam = spec.arrival_peak * (1 - math.cos(2 * math.pi * t / S)) / 2
            cdf = stats.poisson.cdf(np.arange(24), lam) if lam > 0 else np.ones(24)
            assert np.all(np.diff(tp[t].astype(np.int64)) >= 0)
            approx = (tp[t].astype(np.float64) + 1) / 2**32
            assert np.all(np.abs(approx - cdf) <= 2.0**-32 + 1e-13), (t, approx - cdf)


def test_dwell_table_matches_scipy(oracle_lib):
    spec = W.tiny_parity_station()
    c = oracle_lib.OracleClass(spec)
    _, td = c.tables()
    k = np.arange(1, spec.dwell_max)
    F = stats.lognorm.cdf(k + 0.5, s=spec.dwell_sigma, scale=math.exp(spec.dwell_mu))
    approx = (td[1:].astype(np.float64) + 1) / 2**32
    assert np.all(np.diff(td[1:].astype(np.int64)) >= 0)
    assert np.all(np.abs(approx - F) <= 2.0**-32 + 1e-12)


def test_arrivals_statistics(oracle_lib):
    """Mean daily arrivals equal the integral of lambda: 0.3/2 * 288 = 43.2 cars;
    P(M = 0 at step t) equals exp(-lambda(t))."""
    o = oracle_lib
    spec = W.tiny_parity_station().replace(n_levels=10)
    c = o.OracleClass(spec)
    n_env = 1500
    bs = o.BatchState([c], np.zeros(n_env, np.int32))
    out = o.rollout(bs, 11, 288, mode=o.ACT_MAX, want_obs=False, want_act=False, want_info=True)
    M = out["info"]["M"]                          # [288][n_env]
    daily = M.sum(axis=0)
    assert abs(daily.mean() - 43.2) < 4 * math.sqrt(43.2 / n_env)
    t = np.arange(288)
    lam = 0.3 * (1 - np.cos(2 * np.pi * t / 288)) / 2
    p0 = (M == 0).mean(axis=1)
    sd = np.sqrt(np.exp(-lam) * (1 - np.exp(-lam)) / n_env) + 1e-9
    z = (p0 - np.exp(-lam)) / sd
    assert np.abs(z).max() < 5.5
    assert abs(M.var(axis=1).mean() - lam.mean()) < 0.01   # Poisson: variance = mean


def _many_cars(o, n_calls=3000):
    spec = W.tiny_parity_station().replace(arrival_peak=20.0)
    c = o.OracleClass(spec)
    caps, socs, tgts, dw = [], [], [], []
    for i in range(n_calls):
        x = c.draw_exo(99, i % 97, i // 97, 144)
        caps += list(x.car_cap[:x.M])
        socs += list(x.car_soc[:x.M])
        tgts += list(x.car_tgt[:x.M])
        dw += list(x.car_dwell[:x.M])
    return np.array(caps), np.array(socs), np.array(tgts), np.array(dw)


def test_car_profile_statistics(oracle_lib):
    caps, socs, tgts, dw = _many_cars(oracle_lib)
    n = caps.size
    assert n > 40000
    for v, lo, hi in [(caps, 40, 100), (socs, 0.1, 0.5), (tgts, 0.7, 1.0)]:
        assert v.min() >= lo and v.max() < hi
        assert stats.kstest((v - lo) / (hi - lo), "uniform").pvalue > 1e-4
    # dwell: rounded lognormal(ln 36, 0.5), lumped into 1 below 1.5
    k = np.arange(1, 1025)
    F = stats.lognorm.cdf(k + 0.5, s=0.5, scale=36.0)
    F[-1] = 1.0
    pmf = np.diff(np.concatenate([[0.0], F]))
    mean = (k * pmf).sum()
    sd = math.sqrt(((k - mean) ** 2 * pmf).sum())
    assert abs(mean - math.exp(math.log(36) + 0.125)) < 0.05       # ~40.79, rounding barely moves it
    assert abs(dw.mean() - mean) < 5 * sd / math.sqrt(n)
    assert dw.min() >= 1 and abs(np.median(dw) - 36) <= 1
    counts = np.bincount(dw, minlength=1025)[1:]
    exp = pmf * n
    sel = exp > 20
    chi = ((counts[sel] - exp[sel]) ** 2 / exp[sel]).sum()
    assert stats.chi2.sf(chi, sel.sum() - 1) > 1e-4


def test_price_noise_statistics(oracle_lib):
    o = oracle_lib
    c = o.OracleClass(W.tiny_parity_station())
    z = np.array([c.draw_exo(5, e, g, g % 288).z for e in range(40) for g in range(500)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size) and abs(z.std() - 1) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # p_buy = 0.25 + 0.1 sin(2 pi t / 288) + 0.02 z; its daily mean is 0.25
    p = np.array([c.draw_exo(6, e, g, g).p_buy for e in range(30) for g in range(288)])
    assert abs(p.mean() - 0.25) < 5 * 0.02 / math.sqrt(p.size) + 1e-12
    resid = p.reshape(30, 288) - (0.25 + 0.1 * np.sin(2 * np.pi * np.arange(288) / 288))
    assert abs(resid.std() - 0.02) < 0.001


def test_random_actions_steps_independent(oracle_lib):
    """One Philox call serves 8 steps of a port: the levels of steps 1, 2, 4 and
    8 apart (inside a call, across its words, across calls) are independent."""
    o = oracle_lib
    c = o.OracleClass(W.tiny_parity_station())
    ks = np.array([[c.draw_actions(o.ACT_RANDOM, 9, e, g)[0] for g in range(48)] for e in range(400)])
    for lag in (1, 2, 4, 8):
        a, b = ks[:, :-lag].ravel(), ks[:, lag:].ravel()
        table = np.zeros((11, 11))
        np.add.at(table, (a, b), 1)
        assert stats.chi2_contingency(table)[1] > 1e-4, lag


def test_random_actions_uniform(oracle_lib):
    o = oracle_lib
    c = o.OracleClass(W.tiny_parity_station())
    ks = np.concatenate([c.draw_actions(o.ACT_RANDOM, 3, e, g) for e in range(50) for g in range(40)])
    counts = np.bincount(ks, minlength=11)
    assert counts.size == 11
    exp = ks.size / 11
    assert stats.chi2.sf(((counts - exp) ** 2 / exp).sum(), 10) > 1e-4
    assert np.all(c.draw_actions(o.ACT_MAX, 3, 0, 0) == 10)
    ext = np.array([0, 3, 10, 200] * 4, np.uint8)
    assert list(c.draw_actions(o.ACT_EXTERNAL, 3, 0, 0, ext)) == [0, 3, 10, 10] * 4
