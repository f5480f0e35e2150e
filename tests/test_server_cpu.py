"""Serving scheduler on the host clock alone (simulate_ns > 0: every chunk takes
simulate_ns per env-step and nothing touches a GPU): first-come-first-served
admission against the memory budget, refusal of requests that can never fit,
cancellation of queued and running requests, release, and the statistics."""
import time

import numpy as np
import pytest

import workloads as W

NS = 200  # simulated nanoseconds per env-step


@pytest.fixture(scope="module")
def cxm():
    from paper_2507_01522_amd import cx
    return cx


def request_bytes(cxm, spec, n_envs, T, out_mode):
    """Bytes the server charges for a request (read back from a roomy server)."""
    s = cxm.Server(1 << 50, simulate_ns=1)
    t = s.submit(spec, n_envs, T, 1, out_mode)
    r = s.wait(t)
    s.close()
    return int(r.bytes)


def test_bytes_follow_the_layout(cxm):
    spec = W.tiny_parity_station()
    full = request_bytes(cxm, spec, 64, 32, cxm.OUT_FULL)
    rew = request_bytes(cxm, spec, 64, 32, cxm.OUT_REWARD)
    N = spec.n_ports
    rec_full = 64 * 32 * (4 * (6 * N + 4) + N + 4 + 1)
    rec_rew = 64 * 32 * (4 + 1)
    state = 64 * (22 * N + 8)
    # the device block is the class constants + state + server-owned records, each part
    # rounded up to 256 bytes: the difference between the two modes is the records
    assert abs((full - rew) - (rec_full - rec_rew)) <= 4 * 256
    assert rew >= state + rec_rew


def test_fifo_admission_against_budget(cxm):
    spec = W.tiny_parity_station()
    X = request_bytes(cxm, spec, 64, 64, cxm.OUT_FULL)
    small = request_bytes(cxm, spec, 8, 64, cxm.OUT_FULL)
    assert small < X // 2
    s = cxm.Server(int(2.5 * X), chunk_steps=16, max_active=16, simulate_ns=NS)
    a = s.submit(spec, 64, 64, 1, cxm.OUT_FULL)
    b = s.submit(spec, 64, 64, 2, cxm.OUT_FULL)
    c = s.submit(spec, 64, 64, 3, cxm.OUT_FULL)       # does not fit until a release
    d = s.submit(spec, 8, 64, 4, cxm.OUT_FULL)        # would fit, but may not skip ahead of c
    ra, rb = s.wait(a), s.wait(b)
    assert ra.status == 0 and rb.status == 0
    time.sleep(0.05)
    assert s.poll(c) is None and s.poll(d) is None    # still queued: memory is held until release
    s.release(a)
    rc, rd = s.wait(c), s.wait(d)
    assert rc.status == 0 and rd.status == 0
    assert rc.admit_s >= ra.done_s and rd.admit_s >= rc.admit_s
    assert rc.submit_s <= rd.submit_s
    for t in (b, c, d):
        s.release(t)
    st = s.stats()
    assert st["env_steps"] == 3 * 64 * 64 + 8 * 64
    assert st["peak_active"] == 2                     # a and b, then c and d (b had finished)
    assert st["launches"] >= 64 // 16
    s.close()


def test_never_fits_and_invalid(cxm):
    spec = W.tiny_parity_station()
    X = request_bytes(cxm, spec, 64, 64, cxm.OUT_FULL)
    s = cxm.Server(X - 1, simulate_ns=NS)
    with pytest.raises(cxm.CxError) as e:
        s.submit(spec, 64, 64, 1, cxm.OUT_FULL)
    assert e.value.status == -5                        # CX_E_BUDGET
    for bad in [dict(n_envs=0, T=4), dict(n_envs=4, T=0)]:
        with pytest.raises(cxm.CxError) as e:
            s.submit(spec, bad["n_envs"], bad["T"], 1, cxm.OUT_FULL)
        assert e.value.status == -1
    with pytest.raises(cxm.CxError):
        s.submit(spec, 4, 4, 1, cxm.OUT_FULL, act_mode=cxm.ACT_POLICY)
    big = W.fanout4_tree(256, 3)                       # 700,000 x 1540 obs floats: past 2^32 bytes per step
    with pytest.raises(cxm.CxError) as e:
        s.submit(big, 700_000, 4, 1, cxm.OUT_FULL)
    assert e.value.status == -1
    bad_spec = W.single_transformer(8)
    bad_spec.node_limit_kw = np.array([-1.0])
    with pytest.raises(cxm.CxError):
        s.submit(bad_spec, 4, 4, 1, cxm.OUT_FULL)
    with pytest.raises(cxm.CxError) as e:
        s.release(12345)
    assert e.value.status == -7                        # CX_E_NOTFOUND
    s.close()


def test_cancel_queued_and_running(cxm):
    spec = W.tiny_parity_station()
    X = request_bytes(cxm, spec, 1000, 2000, cxm.OUT_REWARD)
    s = cxm.Server(int(1.5 * X), chunk_steps=32, simulate_ns=1000)   # 2 s of simulated work each
    run = s.submit(spec, 1000, 2000, 1, cxm.OUT_REWARD)
    queued = s.submit(spec, 1000, 2000, 2, cxm.OUT_REWARD)
    time.sleep(0.05)
    s.cancel(queued)
    rq = s.wait(queued)
    assert rq.status == -6                             # CX_E_CANCELLED
    s.cancel(run)
    t0 = time.perf_counter()
    rr = s.wait(run)
    assert rr.status == -6 and time.perf_counter() - t0 < 1.0
    st = s.stats()
    assert 0 < st["env_steps"] < 1000 * 2000
    with pytest.raises(cxm.CxError):
        s.poll(12345)
    s.release(queued)
    s.release(run)
    with pytest.raises(cxm.CxError) as e:
        s.poll(run)
    assert e.value.status == -7
    s.close()


def test_release_while_running_is_refused(cxm):
    spec = W.tiny_parity_station()
    s = cxm.Server(1 << 40, chunk_steps=8, simulate_ns=1000)
    t = s.submit(spec, 1000, 1000, 1, cxm.OUT_REWARD)
    with pytest.raises(cxm.CxError) as e:
        s.release(t)
    assert e.value.status == -4                        # CX_E_BUSY
    s.cancel(t)
    s.wait(t)
    s.release(t)
    s.close()


def test_max_active_bounds_concurrency(cxm):
    spec = W.tiny_parity_station()
    s = cxm.Server(1 << 40, chunk_steps=16, max_active=2, simulate_ns=NS)
    ts = [s.submit(spec, 32, 48, i, cxm.OUT_REWARD) for i in range(5)]
    rs = [s.wait(t) for t in ts]
    assert all(r.status == 0 for r in rs)
    assert s.stats()["peak_active"] == 2
    # with two slots, the third request starts only after one of the first two ended
    assert rs[2].admit_s >= min(rs[0].done_s, rs[1].done_s)
    s.close()


def test_blocks_are_contiguous_and_coalesce(cxm):
    """A request needs one contiguous block: two separate free ranges that add up
    to enough do not admit it; releasing the block between them does."""
    spec = W.tiny_parity_station()
    X = request_bytes(cxm, spec, 64, 64, cxm.OUT_FULL)
    D = request_bytes(cxm, spec, 96, 64, cxm.OUT_FULL)
    assert X < D < 2 * X
    s = cxm.Server(3 * X, chunk_steps=16, simulate_ns=NS)
    a, b, c = (s.submit(spec, 64, 64, i, cxm.OUT_FULL) for i in range(3))
    for t in (a, b, c):
        assert s.wait(t).status == 0
    s.release(a)
    s.release(c)                                       # free: [0, X) and [2X, 3X)
    d = s.submit(spec, 96, 64, 9, cxm.OUT_FULL)
    time.sleep(0.05)
    assert s.poll(d) is None                           # 2X free in total, no 1.5X range
    s.release(b)                                       # coalesces into [0, 3X)
    assert s.wait(d).status == 0
    s.release(d)
    s.close()
