"""Serving-loop scheduling on the CPU, through the test-double executor (include/frg_testing.h):
admission against the HBM budget, arrival order, rejection of oversized requests, cancellation,
the watchdog, close-while-busy and the statistics.  No device work runs and nothing is computed;
the result checks of sessions are GPU tests."""
import ctypes
import threading
import time

import numpy as np
import pytest

from paper_2412_13043_amd import frg


def _cfg(inflight=2, budget=1 << 20, poll_us=50, watchdog_ms=0):
    return frg.frg_session_config(inflight, budget, poll_us, watchdog_ms)


class Req:
    """Host buffers of one two-point request (kept alive until its ticket ends)."""

    def __init__(self, n_ext=64, n_q=16, n_x=8):
        self.p = np.linspace(0.01, 5.0, n_ext)
        self.out = np.full(n_ext, -1.0)
        self.desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, n_q, 10.0, n_x=n_x)
        self.batch = frg.frg_batch(n_ext, self.p.ctypes.data, None, 0.5,
                                   frg.frg_log_table(None, 0, 1e-3, 1e3),
                                   self.out.ctypes.data, None)

    @property
    def nodes(self):
        return self.batch.n_ext * self.desc.n_q * self.desc.n_x

    def footprint(self):
        # inputs (p) and outputs, 256-byte aligned pieces (no radial chunks at these sizes, so
        # no contribution block); a launch also holds its request and tile tables, a few KiB
        a = lambda v: (v + 255) // 256 * 256
        n = self.batch.n_ext
        return a(a(n * 8) + a(n * 8))


def test_fake_session_completes_in_arrival_order_with_one_slot():
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=1 << 30), 100.0, 200.0)
    reqs = [Req(n_ext=32 + 8 * i) for i in range(6)]
    tickets = [frg.frg_session_submit(s, r.desc, r.batch, -1) for r in reqs]
    for t in tickets:
        assert frg.frg_session_wait(s, t, 5000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert st.completed == 6 and st.failed == 0 and st.rejected == 0
    assert st.nodes == sum(r.nodes for r in reqs)
    assert st.p50_us > 0 and st.p99_us >= st.p50_us and st.gnodes_per_s > 0
    # the test double never writes outputs
    assert all(np.all(r.out == -1.0) for r in reqs)
    frg.frg_session_close(s)


def test_admission_waits_for_memory_and_never_fails():
    r0 = Req(n_ext=160)
    budget = 2 * r0.footprint() + 4096  # at most two requests (and their tables) fit at once
    s = frg.frg_session_open_fake(_cfg(inflight=4, budget=budget), 2000.0, 1000.0)
    reqs = [Req(n_ext=160) for _ in range(10)]
    t0 = time.perf_counter()
    tickets = [frg.frg_session_submit(s, r.desc, r.batch, -1) for r in reqs]
    st = frg.frg_session_stats(s)
    assert st.queued + st.admitted == 10
    for t in tickets:
        assert frg.frg_session_wait(s, t, 20000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert st.completed == 10 and st.failed == 0
    # at most two requests were resident together, so at least five launches were needed
    assert st.launches >= 5
    assert time.perf_counter() - t0 > 5 * (1e-3 + 2000e-9 * reqs[0].nodes) * 0.9
    frg.frg_session_close(s)


def test_request_larger_than_budget_is_rejected_at_submit():
    big = Req(n_ext=4096, n_q=64)
    s = frg.frg_session_open_fake(_cfg(budget=big.footprint() // 2), 1.0, 1.0)
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_submit(s, big.desc, big.batch, -1)
    assert ei.value.status == frg.FRG_E_NOMEM
    assert frg.frg_session_stats(s).rejected == 1
    frg.frg_session_close(s)


def test_cancel_queued_and_running():
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=1 << 30), 0.0, 300000.0)  # 0.3 s/launch
    a, b = Req(), Req()
    ta = frg.frg_session_submit(s, a.desc, a.batch, -1)
    time.sleep(0.05)  # a is launched, b waits for the only slot
    tb = frg.frg_session_submit(s, b.desc, b.batch, -1)
    assert frg.frg_session_cancel(s, tb) == frg.FRG_OK
    assert frg.frg_session_cancel(s, ta) == frg.FRG_E_NOTREADY
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_wait(s, tb, 1000)
    assert ei.value.status == frg.FRG_E_CANCELLED
    assert frg.frg_session_wait(s, ta, 5000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert st.cancelled == 1 and st.completed == 1
    frg.frg_session_close(s)


def test_wait_timeout_and_watchdog():
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=1 << 30, watchdog_ms=50), 0.0, 400000.0)
    a = Req()
    t = frg.frg_session_submit(s, a.desc, a.batch, -1)
    assert frg.frg_session_wait(s, t, 10) == frg.FRG_E_TIMEOUT  # still running
    time.sleep(0.15)  # the watchdog fails the ticket after 50 ms
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_poll(s, t)
    assert ei.value.status == frg.FRG_E_TIMEOUT
    assert frg.frg_session_stats(s).failed == 1
    frg.frg_session_close(s)  # drains the still-running launch


def test_close_while_busy_cancels_queued():
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=1 << 30), 0.0, 200000.0)
    reqs = [Req() for _ in range(3)]
    tickets = [frg.frg_session_submit(s, r.desc, r.batch, -1) for r in reqs]
    time.sleep(0.02)
    frg.frg_session_close(s)  # the running launch finishes, the two queued ones are cancelled


def test_many_threads_submit_concurrently():
    # one slot and 2 ms per launch: requests arriving during a launch join the next one
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=1 << 30), 0.0, 2000.0)
    errors = []

    def client(i):
        try:
            for k in range(20):
                r = Req(n_ext=16 + (i * 7 + k) % 50)
                t = frg.frg_session_submit(s, r.desc, r.batch, -1)
                assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
        except Exception as e:  # pragma: no cover
            errors.append(e)

    th = [threading.Thread(target=client, args=(i,)) for i in range(16)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    st = frg.frg_session_stats(s)
    assert st.completed == 320 and st.failed == 0
    # continuous batching: launches carried several requests on average
    assert st.launches < 160
    frg.frg_session_close(s)


def test_invalid_session_arguments():
    h = ctypes.c_void_p()
    bad = [_cfg(inflight=0), _cfg(inflight=17), _cfg(budget=100)]
    for c in bad:
        assert frg.raw_status("frg_session_open_fake", ctypes.byref(c), 1.0, 1.0,
                              ctypes.byref(h)) == frg.FRG_E_INVAL
    s = frg.frg_session_open_fake(_cfg(), 1.0, 1.0)
    r = Req()
    with pytest.raises(frg.FrgError):
        frg.frg_session_submit(s, r.desc, r.batch, 5)  # unknown table
    r.desc.n_q = 0
    with pytest.raises(frg.FrgError):
        frg.frg_session_submit(s, r.desc, r.batch, -1)
    with pytest.raises(frg.FrgError):
        frg.frg_session_wait(s, 999, 10)
    Z = np.ones(16)
    tid = frg.frg_session_register_table(s, Z.ctypes.data, 16, 1e-3, 1e3)
    assert tid == 0
    frg.frg_session_close(s)


def test_derivative_outputs_at_submit():
    # sessions return the mass derivative (float64) and the dressing derivatives (float64, with
    # a table: the batch's or a resident one)
    s = frg.frg_session_open_fake(_cfg(), 1.0, 1.0)
    r = Req()
    Z = np.ones(16)
    r.batch.Z = frg.frg_log_table(Z.ctypes.data, 16, 1e-3, 1e3)
    sink = np.zeros(r.batch.n_ext * 16)
    b = frg.frg_batch.from_buffer_copy(r.batch)
    b.dout_dz = sink.ctypes.data
    t = frg.frg_session_submit(s, r.desc, b, -1)
    assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
    tid = frg.frg_session_register_table(s, Z.ctypes.data, 16, 1e-3, 1e3)
    b.Z = frg.frg_log_table(None, 0, 1e-3, 1e3)
    t = frg.frg_session_submit(s, r.desc, b, tid)
    assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
    # without any table: invalid; the float32 form: not implemented
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_submit(s, r.desc, b, -1)
    assert ei.value.status == frg.FRG_E_INVAL
    b.Z = frg.frg_log_table(Z.ctypes.data, 16, 1e-3, 1e3)
    d32 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8, precision=1,
                        near_pole_tau=0.1)
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_submit(s, d32, b, -1)
    assert ei.value.status == frg.FRG_E_UNSUPPORTED
    # dI/dm2 of the float32 form does not exist
    err = np.zeros(r.batch.n_ext)
    b = frg.frg_batch.from_buffer_copy(r.batch)
    b.dout_dm2 = sink.ctypes.data
    b.err_out = err.ctypes.data
    d32 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8, precision=1,
                        near_pole_tau=0.1)
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_submit(s, d32, b, -1)
    assert ei.value.status == frg.FRG_E_UNSUPPORTED
    # float64 with dI/dm2: admitted and completed
    b = frg.frg_batch.from_buffer_copy(r.batch)
    b.dout_dm2 = sink.ctypes.data
    t = frg.frg_session_submit(s, r.desc, b, -1)
    assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
    frg.frg_session_close(s)


def test_mass_derivative_counts_in_the_footprint():
    # the derivative's output array takes device bytes like the values': with launch tables of
    # T <= 32 KiB, a budget of footprint + 32 KiB holds the request without it (it needs
    # footprint + T) but not with it (footprint + 32 KiB + T)
    r = Req(n_ext=4096, n_q=16, n_x=8)
    sink = np.zeros(4096)
    with_d = frg.frg_batch.from_buffer_copy(r.batch)
    with_d.dout_dm2 = sink.ctypes.data
    base = r.footprint()
    extra = 4096 * 8
    s = frg.frg_session_open_fake(_cfg(budget=base + extra + 32768, inflight=2), 1.0, 1.0)
    t = frg.frg_session_submit(s, r.desc, with_d, -1)
    assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
    frg.frg_session_close(s)
    s = frg.frg_session_open_fake(_cfg(budget=base + 32768, inflight=2), 1.0, 1.0)
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_submit(s, r.desc, with_d, -1)
    assert ei.value.status == frg.FRG_E_NOMEM
    t = frg.frg_session_submit(s, r.desc, r.batch, -1)
    assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
    frg.frg_session_close(s)


def _ft_desc(**kw):
    args = dict(n_x=8, T=0.2, freq_max=5.0, statistics=frg.FRG_BOSONIC, n_tail=4)
    args.update(kw)
    return frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 16, 6.0, **args)


def test_finite_temperature_descriptors_are_validated_at_submit():
    s = frg.frg_session_open_fake(_cfg(budget=64 << 20), 1.0, 1.0)
    n = 32
    ext = np.concatenate([np.linspace(0.1, 3.0, n), np.zeros(n)])  # p then p0
    out = np.full(n, -1.0)
    b = frg.frg_batch(n, ext.ctypes.data, None, 0.5, frg.frg_log_table(None, 0, 1e-3, 1e3),
                      out.ctypes.data, None)
    t = frg.frg_session_submit(s, _ft_desc(), b, -1)
    assert frg.frg_session_wait(s, t, 5000) == frg.FRG_OK
    bad = [dict(T=0.0), dict(T=float("nan")), dict(freq_max=-1.0), dict(statistics=2),
           dict(n_tail=-1), dict(n_tail=frg.FRG_MAX_NODES + 1),
           # fermionic with Lambda < pi T: no explicit frequency
           dict(statistics=frg.FRG_FERMIONIC, T=1.0, freq_max=1.0),
           # more than FRG_MAX_NODES frequencies
           dict(T=1e-4, freq_max=10.0),
           # 16 radial nodes x 2000+ frequencies > FRG_MAX_FT_NODES
           dict(T=0.01, freq_max=60.0, n_tail=100)]
    for kw in bad:
        with pytest.raises(frg.FrgError) as ei:
            frg.frg_session_submit(s, _ft_desc(**kw), b, -1)
        assert ei.value.status == frg.FRG_E_INVAL, kw
    d = _ft_desc()
    d.family = 6
    with pytest.raises(frg.FrgError):
        frg.frg_session_submit(s, d, b, -1)
    frg.frg_session_close(s)


def test_footprint_counts_inputs_outputs_and_tables():
    # a finite-temperature request (p and p0 in, I out) needs a(2n*8) + a(n*8) device bytes and
    # no contribution scratch, plus its launch's tables (256 tiles: a few KiB): a budget of that
    # plus 8 KiB admits it, twice the points do not fit
    n, n_q = 256, 16
    a = lambda v: (v + 255) // 256 * 256
    need = a(a(2 * n * 8) + a(n * 8)) + 8192
    s = frg.frg_session_open_fake(_cfg(budget=need), 1.0, 1.0)
    p = np.linspace(0.1, 3.0, n)
    ext = np.concatenate([p, np.zeros(n)])
    out = np.empty(n)
    zt = frg.frg_log_table(None, 0, 1e-3, 1e3)
    bt = frg.frg_batch(n, ext.ctypes.data, None, 0.5, zt, out.ctypes.data, None)
    t = frg.frg_session_submit(s, _ft_desc(), bt, -1)
    assert frg.frg_session_wait(s, t, 5000) == frg.FRG_OK
    # twice the points do not fit
    ext2 = np.concatenate([np.linspace(0.1, 3.0, 2 * n), np.zeros(2 * n)])
    out2 = np.empty(2 * n)
    b2 = frg.frg_batch(2 * n, ext2.ctypes.data, None, 0.5, zt, out2.ctypes.data, None)
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_submit(s, _ft_desc(), b2, -1)
    assert ei.value.status == frg.FRG_E_NOMEM
    frg.frg_session_close(s)


def test_large_request_runs_in_parts_and_small_ones_overtake():
    # a request of 4096 points x 128 x 64 x 16 nodes (5.4e8) runs in parts of at most 2e8 nodes,
    # at most two at a time; two small requests submitted right after it complete before it, on
    # the third slot
    s = frg.frg_session_open_fake(_cfg(inflight=3, budget=1 << 30), 1.0, 100.0)  # 1 ns/node
    n = 4096
    ext = np.concatenate([np.linspace(0.01, 5.0, n), np.linspace(0.0, 3.0, n)])
    out = np.full(n, -1.0)
    big = frg.frg_batch(n, ext.ctypes.data, None, 0.5, frg.frg_log_table(None, 0, 1e-3, 1e3),
                        out.ctypes.data, None)
    dbig = frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 128, 10.0, n_x=64, n_phi=16)
    tb = frg.frg_session_submit(s, dbig, big, -1)
    small = [Req(n_ext=64) for _ in range(2)]
    ts = [frg.frg_session_submit(s, r.desc, r.batch, -1) for r in small]
    for t in ts:
        assert frg.frg_session_wait(s, t, 5000) == frg.FRG_OK
    assert frg.frg_session_poll(s, tb) is False  # 0.54 s of fake work, not done yet
    assert frg.frg_session_wait(s, tb, 10000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert st.completed == 3 and st.failed == 0
    assert st.nodes == n * 128 * 64 * 16 + sum(r.nodes for r in small)
    # the big request needed at least ceil(5.4e8 / 2e8) = 3 launches (the small ones may join
    # one of them)
    assert st.launches >= 3
    frg.frg_session_close(s)


def test_bounded_bypass_of_a_request_blocked_on_memory():
    # budget for one big request or a few small ones: while small requests hold memory, the big
    # one waits; small requests behind it may go ahead, but not forever
    small = Req(n_ext=64)
    big = Req(n_ext=4096)
    budget = big.footprint() + 32768  # with its launch tables
    s = frg.frg_session_open_fake(_cfg(inflight=4, budget=budget), 0.0, 3000.0)  # 3 ms/launch
    first = [Req(n_ext=64) for _ in range(2)]
    t_first = [frg.frg_session_submit(s, r.desc, r.batch, -1) for r in first]
    time.sleep(0.001)
    tb = frg.frg_session_submit(s, big.desc, big.batch, -1)
    later = [Req(n_ext=64) for _ in range(200)]
    t_later = [frg.frg_session_submit(s, r.desc, r.batch, -1) for r in later]
    for t in t_first + [tb] + t_later:
        assert frg.frg_session_wait(s, t, 60000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert st.completed == 203 and st.failed == 0
    frg.frg_session_close(s)


def test_tickets_are_forgotten_once_reported_and_memory_stays_flat():
    s = frg.frg_session_open_fake(_cfg(inflight=4, budget=1 << 30), 0.0, 0.0)
    r = Req(n_ext=16)
    for _ in range(20):
        ts = [frg.frg_session_submit(s, r.desc, r.batch, -1) for _ in range(500)]
        for t in ts:
            assert frg.frg_session_wait(s, t, 10000) == frg.FRG_OK
        assert frg.frg_session_stats(s).tickets_held == 0
    st = frg.frg_session_stats(s)
    assert st.completed == 10000 and st.p50_us >= 0.0 and st.p99_us >= st.p50_us
    # a reported ticket is unknown afterwards
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_poll(s, ts[-1])
    assert ei.value.status == frg.FRG_E_INVAL
    frg.frg_session_close(s)


def test_latency_percentiles_follow_the_launch_time():
    # 2 ms per launch, one slot, requests one at a time: no latency below 2 ms (0.5 % bins);
    # the upper bound is loose, the host may be busy with other tests
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=1 << 30, poll_us=20), 0.0, 2000.0)
    r = Req(n_ext=16)
    for _ in range(30):
        t = frg.frg_session_submit(s, r.desc, r.batch, -1)
        assert frg.frg_session_wait(s, t, 5000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert 1990.0 <= st.p50_us <= 20000.0 and st.p50_us <= st.p99_us <= 200000.0
    frg.frg_session_close(s)


def test_failed_launch_fails_its_tickets_and_frees_memory():
    r = Req(n_ext=300)
    s = frg.frg_session_open_fake(_cfg(inflight=1, budget=r.footprint() + 8192), 0.0, 100.0)
    frg.frg_session_fake_fail_launches(s, 1)
    t = frg.frg_session_submit(s, r.desc, r.batch, -1)
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_session_wait(s, t, 5000)
    assert ei.value.status == frg.FRG_E_DEVICE
    # the budget holds one request: the next one is admitted only if the failed one's block was
    # released
    t2 = frg.frg_session_submit(s, r.desc, r.batch, -1)
    assert frg.frg_session_wait(s, t2, 5000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    assert st.failed == 1 and st.completed == 1 and st.tickets_held == 0
    frg.frg_session_close(s)
    with pytest.raises(frg.FrgError):
        frg.frg_session_fake_fail_launches(0, 1)


def test_replay_harness_on_a_fake_session():
    # open-loop replay: 40 arrivals 1 ms apart on a session whose launches take 0.2 ms; every
    # request completes, none earlier than its launch time, and the wall time spans the trace
    s = frg.frg_session_open_fake(_cfg(inflight=2, budget=1 << 30, poll_us=10), 0.0, 200.0)
    reqs = [Req(n_ext=32), Req(n_ext=48)]
    kinds = []
    for r in reqs:
        kinds.append(frg.frg_replay_kind(r.desc, r.batch.n_ext, r.p.ctypes.data, None, -1, None,
                                         0, 1e-3, 1e3, None))
    m2 = [np.full(r.batch.n_ext, 0.5) for r in reqs]
    for k, v in zip(kinds, m2):
        k.m2 = v.ctypes.data
    times = np.arange(40) * 1000.0
    idx = np.arange(40) % 2
    lat, status, mism, wall = frg.frg_serving_replay(None, s, 0, kinds, times, idx, n_waiters=4)
    assert np.all(status == frg.FRG_OK) and np.all(mism == 0)
    assert np.all(lat >= 200.0) and np.all(lat < 50000.0)
    assert 39000.0 <= wall <= 39000.0 + 60000.0
    assert frg.frg_session_stats(s).completed == 40
    frg.frg_session_close(s)
    # arrivals out of order are rejected
    s = frg.frg_session_open_fake(_cfg(), 0.0, 0.0)
    with pytest.raises(frg.FrgError):
        frg.frg_serving_replay(None, s, 0, kinds, [5.0, 1.0], [0, 1])
    frg.frg_session_close(s)


def test_small_requests_go_first_and_large_ones_leave_a_slot():
    # two slots; a large request (4096 x 128 x 64 x 16 = 5.4e8 nodes, parts of 2e8 at 1 ns/node)
    # may hold only one of them, so small requests submitted after it run on the other slot and
    # finish long before it does
    s = frg.frg_session_open_fake(_cfg(inflight=2, budget=1 << 30), 1.0, 50.0)
    n = 4096
    ext = np.concatenate([np.linspace(0.01, 5.0, n), np.linspace(0.0, 3.0, n)])
    out = np.full(n, -1.0)
    big = frg.frg_batch(n, ext.ctypes.data, None, 0.5, frg.frg_log_table(None, 0, 1e-3, 1e3),
                        out.ctypes.data, None)
    dbig = frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 128, 10.0, n_x=64, n_phi=16)
    t0 = time.perf_counter()
    tb = frg.frg_session_submit(s, dbig, big, -1)
    small = [Req(n_ext=64) for _ in range(20)]
    lat = []
    for r in small:
        t = frg.frg_session_submit(s, r.desc, r.batch, -1)
        assert frg.frg_session_wait(s, t, 5000) == frg.FRG_OK
        lat.append(time.perf_counter() - t0)
    assert frg.frg_session_wait(s, tb, 10000) == frg.FRG_OK
    t_big = time.perf_counter() - t0
    # the large request's three parts take >= 0.54 s one after another on its one slot; all
    # twenty small ones are done within its first part
    assert t_big >= 0.5
    assert max(lat) < 0.2
    frg.frg_session_close(s)


def test_python_session_class_on_the_test_double():
    # the Session wrapper: submit on host arrays, wait, stats, a resident table, context manager
    import numpy as np

    with frg.Session(max_inflight=2, hbm_budget_bytes=64 << 20, fake=(1.0, 5.0)) as s:
        desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 8, 10.0, n_x=4)
        Z = np.ones(16)
        tid = s.register_table(Z, 1e-3, 1e3)
        tickets, outs = [], []
        for i in range(5):
            n = 10 + i
            out = np.zeros(n)
            tickets.append(s.submit(desc, out, ext=np.linspace(0.1, 1.0, n), m2_scalar=0.5,
                                    table_id=tid if i % 2 else -1, Z=None if i % 2 else Z))
            outs.append(out)
        for t in tickets:
            assert s.wait(t, 10000) == frg.FRG_OK
        st = s.stats()
        assert st.completed == 5 and st.failed == 0
        with pytest.raises(ValueError):
            s.submit(desc, np.zeros(4, dtype=np.float32), ext=np.ones(4), m2_scalar=0.5)
