"""Host-side admission logic of the continuous-batching server (no GPU)."""
import numpy as np
import pytest

from paper_2411_09982_amd.serve import (Admission, Request, Result, job_bytes, latency_percentiles, max_overlap,
                                         path_for, poisson_requests)


def test_fifo_budget_and_slots():
    a = Admission(budget_bytes=100, max_slots=2)
    for rid, nb in [(0, 40), (1, 50), (2, 30), (3, 5)]:
        a.offer(rid, nb)
    assert a.admit() == [0, 1]          # slot limit
    assert a.in_use == 90
    a.release(0)
    assert a.admit() == [2]             # 50 + 30 <= 100
    assert a.admit() == []              # both slots busy even though 3 would fit
    a.release(1)
    assert a.admit() == [3]
    a.release(2)
    a.release(3)
    assert a.in_use == 0 and not a.running


def test_head_of_line_waits_for_memory():
    a = Admission(budget_bytes=100, max_slots=8)
    a.offer(0, 70)
    a.offer(1, 60)
    a.offer(2, 10)
    assert a.admit() == [0]             # 1 does not fit; 2 does not overtake it
    a.release(0)
    assert a.admit() == [1, 2]


def test_oversized_request_rejected():
    a = Admission(budget_bytes=10, max_slots=1)
    with pytest.raises(ValueError):
        a.offer(0, 11)


def test_job_bytes_accounting():
    d, K, M = 100, 2, 40
    b64 = job_bytes(d, K, M, 2, "c64", 16)
    b128 = job_bytes(d, K, M, 2, "c128", 16)
    # complex64 generators (8 B) plus the refined complex128 propagators (16 B)
    # against complex128 generators overwritten in place by U (16 B)
    assert b64 - b128 == M * d * d * 8
    # the action holds one chunk of generators and no propagators
    a64 = job_bytes(d, K, M, 2, "c64", 16, path="action")
    a128 = job_bytes(d, K, M, 2, "c128", 16, path="action")
    assert a128 - a64 == 16 * d * d * 8
    assert job_bytes(d, K, M, 2, "c64", 16, lambda *a: 1000) == b64 + 1000


def test_poisson_arrivals_deterministic():
    def make(i, g):
        return Request(i, np.eye(2, dtype=complex), np.eye(2, dtype=complex)[None], np.zeros((1, 4)), 0.1, 2, 1,
                       "c64", np.array([1, 0], dtype=complex))
    r1 = poisson_requests(50, 100.0, 7, make)
    r2 = poisson_requests(50, 100.0, 7, make)
    t = np.array([r.arrival for r in r1])
    assert np.all(np.diff(t) > 0) and np.allclose(t, [r.arrival for r in r2])
    assert 0.2 < t[-1] < 1.0            # 50 arrivals at 100 /s


def test_latency_split_into_wait_and_service():
    res = {i: Result(i, np.zeros(1), 0, arrival=0.0, admitted=0.1 * i, done=0.1 * i + 1.0) for i in range(5)}
    lat = latency_percentiles(res)
    assert lat["n"] == 5
    assert lat["service_p50_ms"] == pytest.approx(1000.0) and lat["service_p99_ms"] == pytest.approx(1000.0)
    assert lat["wait_p50_ms"] == pytest.approx(200.0)
    assert lat["p50_ms"] == pytest.approx(1200.0)
    assert lat["p99_ms"] == pytest.approx(1000.0 + 0.99 * 400.0)
    assert max_overlap(res) == 5


def test_path_choice_and_action_memory():
    def req(d, path="auto"):
        return Request(0, np.eye(d, dtype=complex), np.eye(d, dtype=complex)[None], np.zeros((1, 8)), 0.1, 4, 1,
                       "c64", np.eye(d, dtype=complex)[0], path=path)
    assert path_for(req(32)) == "propagators" and path_for(req(33)) == "action"
    assert path_for(req(500, "propagators")) == "propagators" and path_for(req(8, "action")) == "action"
    # the action holds one chunk of generators, the propagators all M of them
    # (complex64) and all M refined propagators (complex128)
    d, K, M, chunk = 100, 2, 40, 8
    assert (job_bytes(d, K, M, 2, "c64", chunk, path="propagators") - job_bytes(d, K, M, 2, "c64", chunk, path="action")
            == (M - chunk) * d * d * 8 + M * d * d * 16)
