"""Scheduler of the render server, on the CPU with a fake executor: admission
by memory budget, arrival order, continuous batching while work is in flight,
failure isolation, oversized requests refused."""
import threading
import time

import pytest

from paper_2509_13536_amd.serve import RenderServer


class FakeView:
    def __init__(self, W, H):
        self.W, self.H = W, H
        self.fx = self.fy = 1.0
        self.cx = self.cy = 0.0
        self.Tcw = None
        self.near = 0.2
        self.map = 0


class FakeExecutor:
    def __init__(self, n_workers=2, delay=0.01, bytes_per_px=10, fail_map=None):
        self.streams = [None] * n_workers
        self.delay = delay
        self.bpp = bytes_per_px
        self.fail_map = fail_map
        self.lock = threading.Lock()
        self.active_bytes = 0
        self.max_active = 0
        self.batches = []
        self.concurrent = 0
        self.max_concurrent = 0

    def estimate_bytes(self, req):
        return self.bpp * req.view.W * req.view.H

    def run(self, worker, batch):
        need = sum(self.estimate_bytes(r) for r in batch)
        with self.lock:
            self.active_bytes += need
            self.max_active = max(self.max_active, self.active_bytes)
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
            self.batches.append([r.rid for r in batch])
        time.sleep(self.delay)
        with self.lock:
            self.active_bytes -= need
            self.concurrent -= 1
        if self.fail_map is not None and any(r.map_id == self.fail_map for r in batch):
            raise RuntimeError("poisoned batch")
        return [("rgb%d" % r.rid, "depth%d" % r.rid) for r in batch]


def test_all_requests_complete_in_order_within_budget():
    ex = FakeExecutor(n_workers=2, delay=0.005)
    budget = 10 * 100 * 100 * 6  # six 100x100 requests
    srv = RenderServer(ex, budget, max_batch=4)
    futs = [srv.submit(0, FakeView(100, 100)) for _ in range(40)]
    res = [f.result(timeout=30) for f in futs]
    srv.close()
    assert [r.rgb for r in res] == ["rgb%d" % i for i in range(40)]
    assert ex.max_active <= budget
    flat = [rid for b in ex.batches for rid in b]
    assert sorted(flat) == list(range(40))
    # batches are admitted in arrival order: each batch is a run of consecutive
    # arrivals, and the runs tile the stream (concurrent workers may start
    # their batches in either order)
    runs = sorted(ex.batches)
    assert all(b == list(range(b[0], b[0] + len(b))) for b in runs)
    assert [rid for b in runs for rid in b] == list(range(40))
    assert max(len(b) for b in ex.batches) <= 4
    st = srv.stats()
    assert st["completed"] == 40 and st["p99_ms"] >= st["p50_ms"] > 0


def test_budget_below_one_batch_queues_instead_of_deadlocking():
    ex = FakeExecutor(n_workers=3, delay=0.002)
    budget = 10 * 64 * 64  # exactly one request at a time
    srv = RenderServer(ex, budget, max_batch=8)
    futs = [srv.submit(0, FakeView(64, 64)) for _ in range(12)]
    for f in futs:
        f.result(timeout=30)
    srv.close()
    assert ex.max_active <= budget
    assert all(len(b) == 1 for b in ex.batches)


def test_work_overlaps_and_late_arrivals_join_next_batches():
    ex = FakeExecutor(n_workers=2, delay=0.05)
    srv = RenderServer(ex, 10 ** 9, max_batch=16)
    futs = [srv.submit(0, FakeView(10, 10)) for _ in range(3)]
    time.sleep(0.01)  # first batch is on a worker
    futs += [srv.submit(0, FakeView(10, 10)) for _ in range(5)]
    for f in futs:
        f.result(timeout=30)
    srv.close()
    assert ex.max_concurrent == 2
    assert len(ex.batches) >= 2


def test_failing_batch_fails_only_its_requests_and_oversize_is_refused():
    ex = FakeExecutor(n_workers=1, delay=0.001, fail_map=7)
    srv = RenderServer(ex, 10 * 50 * 50 * 2, max_batch=1)
    good = srv.submit(0, FakeView(50, 50))
    bad = srv.submit(7, FakeView(50, 50))
    good2 = srv.submit(0, FakeView(50, 50))
    huge = srv.submit(0, FakeView(500, 500))
    assert good.result(timeout=30).rgb.startswith("rgb")
    assert good2.result(timeout=30).rgb.startswith("rgb")
    with pytest.raises(RuntimeError):
        bad.result(timeout=30)
    with pytest.raises(MemoryError):
        huge.result(timeout=1)
    srv.close()


def test_invalid_request_is_refused_alone():
    """A request the library would refuse (here a NaN pose) fails by itself at
    submit; the requests around it complete."""
    ex = FakeExecutor(n_workers=1, delay=0.001)
    srv = RenderServer(ex, 10 * 50 * 50 * 8, max_batch=8)
    bad_view = FakeView(50, 50)
    bad_view.Tcw = [[float("nan")] * 4] * 3
    zero_f = FakeView(50, 50)
    zero_f.fx = 0.0
    futs = [srv.submit(0, FakeView(50, 50)), srv.submit(0, bad_view), srv.submit(0, zero_f), srv.submit(0, FakeView(50, 50))]
    assert futs[0].result(timeout=30).rgb.startswith("rgb")
    assert futs[3].result(timeout=30).rgb.startswith("rgb")
    for f in futs[1:3]:
        with pytest.raises(ValueError):
            f.result(timeout=1)
    srv.close()


def test_batches_run_on_persistent_workers():
    """Every batch runs on one of n_workers long-lived threads (no thread per
    batch), and the workers end with the server."""
    ex = FakeExecutor(n_workers=3, delay=0.01)
    callers = set()
    run = ex.run

    def recording_run(worker, batch):
        callers.add(threading.get_ident())
        return run(worker, batch)

    ex.run = recording_run
    srv = RenderServer(ex, 10 ** 9, max_batch=2)
    futs = []
    for _ in range(8):  # bursts of three batches: all three workers busy at once
        futs += [srv.submit(0, FakeView(8, 8)) for _ in range(6)]
        time.sleep(0.03)
    for f in futs:
        f.result(timeout=30)
    assert len(ex.batches) >= 24
    workers = list(srv.workers)
    assert callers == {t.ident for t in workers}
    srv.close()
    assert not any(t.is_alive() for t in workers)
