"""Serving loop logic on the CPU with fake executors (no GPU).

Covers admission under the HBM budget, rejection of oversized requests, FIFO
admission, continuous batching (arrivals during a running batch join the next
one), the bound on a batch's cost, overlap of batches on several streams,
failure isolation, and delivery of correct images (an executor that
reconstructs with the FP64 oracle).
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2109_02174_amd import phantom as ph
from paper_2109_02174_amd._binding import Geometry
from paper_2109_02174_amd.serve import Executor, RequestTooLarge, Server, footprint_bytes, request_cost


class FakeSino:
    def __init__(self, n):
        self.shape = (n,)


class SleepExecutor(Executor):
    """Each batch 'runs' for a fixed time on a timer thread; records concurrency."""

    def __init__(self, n_streams=2, run_s=0.05, fail_rid=None, fail_wait_rid=None):
        self.n_streams = n_streams
        self.run_s = run_s
        self.fail_rid = fail_rid
        self.fail_wait_rid = fail_wait_rid
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.batches = []

    def allocate_output(self, req):
        return np.zeros((req.n_slices, 1))

    def launch(self, s, reqs):
        rids = [r.rid for r in reqs]
        if self.fail_rid is not None and self.fail_rid in rids:
            raise RuntimeError("injected launch failure")
        done = threading.Event()
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.batches.append((s, rids))

        def finish():
            with self.lock:
                self.active -= 1
            done.set()
        threading.Timer(self.run_s, finish).start()
        return (done, rids)

    def wait(self, handle):
        done, rids = handle
        done.wait()
        if self.fail_wait_rid is not None and self.fail_wait_rid in rids:
            raise RuntimeError("injected execution failure")


def _geom(K=10, D=15, N=8):
    return Geometry(K, D, N)


def test_all_requests_complete_with_latency():
    ex = SleepExecutor(run_s=0.01)
    srv = Server(ex, hbm_budget_bytes=1 << 30)
    futs = [srv.submit(_geom(), FakeSino(3)) for _ in range(20)]
    assert srv.drain(timeout=10)
    for f in futs:
        assert f.result(timeout=1).shape == (3, 1)
    st = srv.stats()
    assert st["completed"] == 20 and st["slices"] == 60 and st["failed"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    srv.shutdown()


def test_budget_is_respected_and_oversize_rejected():
    g = _geom()
    one = footprint_bytes(g.n_angles, g.n_det, g.image_size, 4)
    ex = SleepExecutor(run_s=0.02)
    srv = Server(ex, hbm_budget_bytes=3 * one)
    big = srv.submit(g, FakeSino(100))
    with pytest.raises(RequestTooLarge):
        big.result(timeout=1)
    futs = [srv.submit(g, FakeSino(4)) for _ in range(12)]
    assert srv.drain(timeout=10)
    assert all(f.done() and f.exception() is None for f in futs)
    assert srv.stats()["max_in_use_bytes"] <= 3 * one
    srv.shutdown()


def test_fifo_admission_under_tight_budget():
    g = _geom()
    one = footprint_bytes(g.n_angles, g.n_det, g.image_size, 2)
    ex = SleepExecutor(n_streams=2, run_s=0.01)
    srv = Server(ex, hbm_budget_bytes=one)       # room for one request at a time
    order = []
    lock = threading.Lock()
    futs = []
    for i in range(8):
        f = srv.submit(g, FakeSino(2))
        f.add_done_callback(lambda _f, i=i: (lock.acquire(), order.append(i), lock.release()))
        futs.append(f)
    assert srv.drain(timeout=10)
    assert order == list(range(8))
    srv.shutdown()


def test_arrivals_during_a_batch_join_the_next_batch():
    ex = SleepExecutor(n_streams=1, run_s=0.2)
    srv = Server(ex, hbm_budget_bytes=1 << 30)
    first = srv.submit(_geom(), FakeSino(1))
    time.sleep(0.05)                              # first batch is now running
    rest = [srv.submit(_geom(), FakeSino(1)) for _ in range(6)]
    assert srv.drain(timeout=10)
    assert len(ex.batches) == 2                   # [first], [the six that arrived meanwhile]
    assert len(ex.batches[0][1]) == 1
    assert len(ex.batches[1][1]) == 6
    assert all(f.exception() is None for f in rest + [first])
    srv.shutdown()


def test_batch_cost_is_bounded_and_order_kept():
    """A queue of admitted requests is cut into batches of at most max_batch_cost
    updates (in arrival order); a request costlier than the bound runs alone."""
    g = _geom()
    unit = request_cost(g.n_angles, g.image_size, 1)
    ex = SleepExecutor(n_streams=1, run_s=0.2)
    srv = Server(ex, hbm_budget_bytes=1 << 30, max_batch_cost=5 * unit)
    first = srv.submit(g, FakeSino(1))
    time.sleep(0.05)                              # the rest queue behind the first batch
    sizes = [2, 2, 2, 9, 1, 3, 1, 1]
    futs = [srv.submit(g, FakeSino(n)) for n in sizes]
    assert srv.drain(timeout=20)
    assert all(f.exception() is None for f in futs + [first])
    got = [[r - 1 for r in rids] for _, rids in ex.batches[1:]]   # request ids of the queued ones
    assert got == [[0, 1], [2], [3], [4, 5, 6], [7]]
    for b in got:
        assert sum(sizes[i] for i in b) * unit <= 5 * unit or len(b) == 1
    srv.shutdown()


def test_batches_overlap_on_several_streams():
    ex = SleepExecutor(n_streams=3, run_s=0.15)
    srv = Server(ex, hbm_budget_bytes=1 << 30, max_batch_slices=2)
    futs = [srv.submit(_geom(), FakeSino(2)) for _ in range(6)]
    assert srv.drain(timeout=10)
    assert ex.max_active >= 2
    assert {s for s, _ in ex.batches} == {0, 1, 2}
    srv.shutdown()


def test_launch_failure_fails_only_its_batch_and_frees_budget():
    g = _geom()
    one = footprint_bytes(g.n_angles, g.n_det, g.image_size, 1)
    ex = SleepExecutor(n_streams=1, run_s=0.01, fail_rid=0)
    srv = Server(ex, hbm_budget_bytes=one, max_batch_slices=1)
    f0 = srv.submit(g, FakeSino(1))
    others = [srv.submit(g, FakeSino(1)) for _ in range(4)]
    assert srv.drain(timeout=10)
    with pytest.raises(RuntimeError):
        f0.result(timeout=1)
    assert all(f.exception() is None for f in others)
    assert srv.stats()["failed"] == 1
    srv.shutdown()


def test_execution_failure_is_reported_and_memory_returned():
    g = _geom()
    ex = SleepExecutor(n_streams=2, run_s=0.01, fail_wait_rid=1)
    srv = Server(ex, hbm_budget_bytes=1 << 30, max_batch_slices=1)
    futs = [srv.submit(g, FakeSino(1)) for _ in range(5)]
    assert srv.drain(timeout=10)
    assert isinstance(futs[1].exception(), RuntimeError)
    assert all(futs[i].exception() is None for i in (0, 2, 3, 4))
    assert srv._in_use == 0
    srv.shutdown()


class OracleExecutor(Executor):
    """Reconstructs each batch with the FP64 oracle on a worker thread."""
    n_streams = 2

    def allocate_output(self, req):
        g = req.geom
        return np.zeros((req.n_slices, g.image_size, g.image_size))

    def launch(self, s, reqs):
        done = threading.Event()

        def run():
            for r in reqs:
                r.output[:] = oracle.fbp(r.sino, r.geom.image_size, r.geom.det_spacing, r.geom.angles)
            done.set()
        threading.Thread(target=run).start()
        return done

    def wait(self, handle):
        handle.wait()


def test_served_images_are_the_reconstructions():
    srv = Server(OracleExecutor(), hbm_budget_bytes=1 << 30)
    cases = []
    for i, (N, K, D) in enumerate([(16, 20, 25), (9, 7, 15), (16, 20, 25)]):
        g = Geometry(K, D, N)
        sino = np.stack([ph.ellipse_slice(77, 3 * i + b, N, K, D, n_ellipses=3).sino for b in range(2)])
        cases.append((g, sino, srv.submit(g, sino)))
    assert srv.drain(timeout=30)
    for g, sino, f in cases:
        assert np.array_equal(f.result(), oracle.fbp(sino, g.image_size, g.det_spacing, g.angles))
    srv.shutdown()
