"""Host logic of the scene-fit server (admission by HBM budget, slots, FIFO,
latency bookkeeping) with fake fits: no GPU involved."""
import threading
import time

import pytest

from paper_2602_00395_amd.serve import FitRequest, Server


def _req(rid, arrival, nbytes, dur):
    r = FitRequest(rid=rid, arrival_s=arrival, n=1000 * (rid + 1), sh_degree=0, make_scene=None, train_ids=[0],
                   test_ids=[0], target_psnr=0.0, bytes_needed=nbytes)
    r.dur = dur
    return r


def test_admission_never_exceeds_budget_and_all_complete():
    live = {"bytes": 0, "peak": 0}
    lock = threading.Lock()

    def fake_fit(req, stream, keep, tf):
        with lock:
            live["bytes"] += req.bytes_needed
            live["peak"] = max(live["peak"], live["bytes"])
        time.sleep(req.dur)
        with lock:
            live["bytes"] -= req.bytes_needed
        return 10, 30.0, True, None

    reqs = [_req(i, 0.01 * i, 300 + 100 * (i % 3), 0.05 + 0.01 * (i % 4)) for i in range(12)]
    srv = Server(hbm_budget=1000, max_active=8, stream_factory=lambda: None)
    st = srv.run(reqs, fit_fn=fake_fit)
    assert len(st.results) == 12 and all(r.reached for r in st.results)
    assert live["peak"] <= 1000 and st.peak_bytes <= 1000
    assert st.peak_bytes >= 700  # the budget is actually used for overlap
    for r in st.results:
        assert r.start_s >= r.arrival_s - 1e-6 and r.end_s >= r.start_s
    # FIFO admission: start times follow arrival order
    starts = [r.start_s for r in sorted(st.results, key=lambda r: r.arrival_s)]
    assert starts == sorted(starts)
    assert st.percentile(50) <= st.percentile(99)
    assert st.gaussian_updates_per_s() > 0


def test_slot_limit_and_oversized_request():
    active = {"now": 0, "max": 0}
    lock = threading.Lock()

    def fake_fit(req, stream, keep, tf):
        with lock:
            active["now"] += 1
            active["max"] = max(active["max"], active["now"])
        time.sleep(0.03)
        with lock:
            active["now"] -= 1
        return 1, 0.0, False, None

    reqs = [_req(i, 0.0, 1, 0.03) for i in range(9)]
    st = Server(hbm_budget=100, max_active=3, stream_factory=lambda: None).run(reqs, fit_fn=fake_fit)
    assert active["max"] <= 3 and len(st.results) == 9
    with pytest.raises(ValueError):
        Server(hbm_budget=10, stream_factory=lambda: None).run([_req(0, 0.0, 11, 0.0)], fit_fn=fake_fit)


def test_failed_fit_is_recorded_and_counts_against_latency():
    def fake_fit(req, stream, keep, tf):
        time.sleep(0.01)
        if req.rid == 2:
            raise RuntimeError("device lost")
        return 5, 25.0, True, None

    reqs = [_req(i, 0.0, 10, 0.01) for i in range(4)]
    st = Server(hbm_budget=100, max_active=2, stream_factory=lambda: None).run(reqs, fit_fn=fake_fit)
    assert len(st.results) == 4
    assert [r.rid for r in st.failed] == [2] and "device lost" in st.failed[0].error
    assert not st.failed[0].reached
    # a failure is an unfinished request: the p99 over 4 requests then is not finite
    assert st.percentile(99) == float("inf")
    assert st.percentile(25) < 1.0
