"""The serving scheduler on the host-only executor (no GPU): admission by budget,
arrival order, back-pressure, cancellation, statistics and shutdown."""
import threading
import time

import numpy as np
import pytest

lp = pytest.importorskip("paper_1204_0556_amd")


def server(**kw):
    kw.setdefault("code_n", [96, 2640])
    return lp.Server(executor=lp.EXECUTOR_HOST_NULL, **kw)


def frames(code_n, k):
    return np.zeros((k, code_n), np.float32)


def test_requests_complete_and_stats_add_up():
    s = server(budget_bytes=1 << 20)
    tickets = [s.submit(i % 2, frames(s.n[i % 2], 1 + i % 5)) for i in range(40)]
    total_bits = sum((1 + i % 5) * s.n[i % 2] for i in range(40))
    for t in tickets:
        x, it, fl, lat = s.wait(t, timeout=5.0)
        assert np.all(x == 0.5) and lat >= 0.0
    st = s.stats()
    assert st["submitted"] == st["completed"] == 40
    assert st["bits_completed"] == total_bits
    assert 0.0 <= st["p50_latency_s"] <= st["p99_latency_s"] <= st["max_latency_s"]
    assert st["inflight_bytes"] == 0
    # the host-only executor has no launch scratch: the device footprint is the arena's
    assert st["workspace_bytes"] == 0 and st["peak_device_bytes"] == st["peak_bytes"]
    assert st["peak_concurrent_launches"] >= 1
    s.close()


def test_budget_is_never_exceeded():
    budget = 2640 * 4 * 3  # three n=2640 frames
    s = server(budget_bytes=budget)
    tickets = []
    for i in range(30):
        tickets.append(s.submit(1, frames(2640, 1 + i % 3)))
    # collect in order; the scheduler must keep the admitted footprint <= budget
    for t in tickets:
        s.wait(t, timeout=5.0)
    st = s.stats()
    assert st["completed"] == 30
    assert 0 < st["peak_bytes"] <= budget


def test_oversized_request_is_rejected():
    s = server(budget_bytes=96 * 4 * 4)
    with pytest.raises(lp.LpdecError) as e:
        s.submit(0, frames(96, 5))
    assert e.value.status == -1 and "exceeds the server budget" in str(e.value)
    assert s.stats()["rejected"] == 1


def test_uncollected_results_apply_back_pressure_and_cancel():
    s = server(budget_bytes=96 * 4 * 2)
    a = s.submit(0, frames(96, 2))  # fills the result arena until collected
    deadline = time.time() + 5
    while s.poll(a) != lp.REQ_DONE and time.time() < deadline:
        time.sleep(0.001)
    b = s.submit(0, frames(96, 2))
    time.sleep(0.01)
    assert s.poll(b) == lp.REQ_QUEUED  # waits for a's results to be collected
    s.cancel(b)
    with pytest.raises(lp.LpdecError):
        s.poll(b)
    c = s.submit(0, frames(96, 1))
    s.wait(a)
    s.wait(c, timeout=5.0)
    assert s.stats()["cancelled"] == 1


def test_admitted_request_cannot_be_cancelled():
    s = server(budget_bytes=1 << 20)
    a = s.submit(0, frames(96, 1))
    deadline = time.time() + 5
    while s.poll(a) == lp.REQ_QUEUED and time.time() < deadline:
        time.sleep(0.001)
    with pytest.raises(lp.LpdecError) as e:
        s.cancel(a)
    assert e.value.status == -5


def test_pending_queue_limit():
    s = server(budget_bytes=96 * 4, max_pending=2)
    first = s.submit(0, frames(96, 1))  # admitted, result held
    deadline = time.time() + 5
    while s.poll(first) != lp.REQ_DONE and time.time() < deadline:
        time.sleep(0.001)
    s.submit(0, frames(96, 1))
    s.submit(0, frames(96, 1))
    with pytest.raises(lp.LpdecError) as e:
        s.submit(0, frames(96, 1))
    assert e.value.status == -5
    s.close()  # drops the queued requests without hanging


def test_wait_timeout_and_unknown_ticket():
    s = server(budget_bytes=96 * 4)
    a = s.submit(0, frames(96, 1))
    deadline = time.time() + 5
    while s.poll(a) != lp.REQ_DONE and time.time() < deadline:
        time.sleep(0.001)
    b = s.submit(0, frames(96, 1))  # blocked behind a's uncollected result
    with pytest.raises(lp.LpdecError) as e:
        s.wait(b, timeout=0.01)
    assert e.value.status == -5
    s.wait(a)
    s.wait(b, timeout=5.0)
    with pytest.raises(lp.LpdecError):
        s.poll(12345)


def test_concurrent_submitters():
    s = server(budget_bytes=1 << 16)
    results = []

    def worker(k):
        for i in range(20):
            t = s.submit(k % 2, frames(s.n[k % 2], 1))
            results.append(s.wait(t, timeout=10.0)[0].shape)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(results) == 80 and s.stats()["completed"] == 80


def test_bad_configuration():
    with pytest.raises(lp.LpdecError):
        lp.Server(code_n=[96], executor=lp.EXECUTOR_HOST_NULL, max_inflight=0)
    with pytest.raises(lp.LpdecError):
        lp.Server(code_n=[96], executor=lp.EXECUTOR_HOST_NULL, budget_bytes=0)
    with pytest.raises(lp.LpdecError):
        lp.Server(code_n=[96], executor=lp.EXECUTOR_GPU)  # the GPU executor needs codes
