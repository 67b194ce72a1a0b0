"""Host logic of the frame server, on the CPU with a fake backend.

Checks that frames of one stream never overlap and run in order, that the
worker-slot and memory budgets are respected, that frames of different
streams do overlap, and that a failing frame is reported without stopping
the server.
"""
import threading
import time

from paper_2410_17084_amd import serve


class FakeBackend(serve.Backend):
    def __init__(self, delay=0.004, fail=None):
        self.delay = delay
        self.fail = fail or set()
        self.lock = threading.Lock()
        self.active = {}
        self.overlap_streams = 0
        self.concurrent = 0
        self.max_concurrent = 0
        self.order = {}

    def update(self, stream, index):
        with self.lock:
            assert stream not in self.active, "two frames of one stream in flight"
            self.active[stream] = index
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
            if len(self.active) > 1:
                self.overlap_streams += 1
            self.order.setdefault(stream, []).append(index)
        time.sleep(self.delay)
        with self.lock:
            del self.active[stream]
            self.concurrent -= 1
        if (stream, index) in self.fail:
            raise RuntimeError("injected failure")
        return 7


def test_order_slots_overlap():
    be = FakeBackend()
    sizes = [[1000, 2000]] * 6
    st = serve.serve(be, sizes, rate_hz=50.0, duration_s=0.4, workers=3, budget_bytes=1 << 40, m=64)
    s = st.summary()
    assert s["frames"] == 6 * 20 and s["failed"] == 0
    for stream, idx in be.order.items():
        assert idx == sorted(idx)
    assert be.max_concurrent <= 3 and st.max_inflight <= 3
    assert be.overlap_streams > 0
    assert s["solves"] == 7 * 6 * 20
    assert s["p50_ms"] is not None and s["p99_ms"] >= s["p50_ms"]


def test_memory_budget_limits_inflight():
    be = FakeBackend(delay=0.003)
    m = 64
    one = serve.working_set_bytes(1000, m)
    st = serve.serve(be, [[1000]] * 4, rate_hz=100.0, duration_s=0.2, workers=4, budget_bytes=2 * one, m=m)
    assert st.max_inflight_bytes <= 2 * one
    assert be.max_concurrent <= 2


def test_oversized_frame_still_admitted_alone():
    be = FakeBackend(delay=0.001)
    st = serve.serve(be, [[10 ** 6]], rate_hz=20.0, duration_s=0.2, workers=2, budget_bytes=1, m=64)
    assert st.summary()["frames"] == 4 and st.max_inflight == 1


def test_failure_is_reported_and_server_continues():
    be = FakeBackend(fail={(1, 2)})
    st = serve.serve(be, [[100]] * 3, rate_hz=50.0, duration_s=0.2, workers=2, budget_bytes=1 << 40, m=16)
    s = st.summary()
    assert s["failed"] == 1 and s["frames"] == 30
    bad = [r for r in st.requests if r.error]
    assert (bad[0].stream, bad[0].index) == (1, 2)


def test_backlog_mode_and_stream_subset():
    be = FakeBackend(delay=0.001)
    st = serve.serve(be, [[10]] * 4, rate_hz=10.0, duration_s=1.0, workers=4, budget_bytes=1 << 40, m=16,
                     streams=[2], realtime=False)
    assert {r.stream for r in st.requests} == {2} and len(st.requests) == 10
