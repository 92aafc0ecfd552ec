"""The serving loop's scheduling on the CPU, with a fake executor whose
batches complete after a modelled time: every request completes once, FIFO
admission, the arena never overflows, batches overlap (continuous batching),
a batch that finishes before an earlier one is recorded and freed at once,
admission charges the full footprint (24 N L bytes plus workspace),
oversize requests are rejected, a tiny budget forces queueing."""
import time

import numpy as np
import pytest

from paper_2209_01290_amd import serve, workloads


class FakeExecutor:
    """Batches complete `us_per_product` microseconds per N = 2^16 limb-product
    after launch (or at the time `finish_at(batch)` gives, when set)."""

    def __init__(self, us_per_product=20.0, finish_at=None):
        self.us = us_per_product
        self.finish_at = finish_at
        self.launched = []
        self.blocks = []

    def launch(self, batch, k, block):
        dur = self.us * 1e-6 * sum(r.limbs * (1 << r.log2n) / 65536.0 for r in batch)
        now = time.monotonic()
        self.launched.append((now, [r.rid for r in batch]))
        self.blocks.append(block)
        return self.finish_at(batch, now) if self.finish_at else now + dur

    def done(self, handle):
        return time.monotonic() >= handle

    def finish(self, handle):
        pass


def _one(tr):
    """Arena bytes that hold the largest request of a trace in a batch of its own."""
    return max(serve.request_bytes(n, L) for _, n, L in tr) + serve.BATCH_WS_SLACK


def _trace(n, rate, seed=1):
    return workloads.serving_requests(seed, n, rate)


def test_trace_distribution():
    tr = _trace(20000, 10000.0)
    t = np.array([x[0] for x in tr])
    gaps = np.diff(t)
    assert abs(gaps.mean() * 10000.0 - 1.0) < 0.05          # Poisson at the requested rate
    ns = np.array([x[1] for x in tr])
    for log2n, w in zip(workloads.SERVE_LOG2N, workloads.SERVE_WEIGHTS):
        assert abs((ns == log2n).mean() - w) < 0.02
    Ls = np.array([x[2] for x in tr])
    assert Ls.min() == 1 and Ls.max() == 60 and abs(Ls.mean() - 30.5) < 1.0


def test_every_request_completes_fifo():
    ex = FakeExecutor()
    eng = serve.Engine(ex, budget_bytes=8 << 30, streams=3)
    st = eng.run(_trace(400, 20000.0))
    reqs = st["_requests"]
    assert st["completed"] == 400 and st["rejected"] == 0
    admits = [r.t_admit for r in reqs]
    assert all(a <= b for a, b in zip(admits, admits[1:]))           # FIFO admission
    assert all(r.t_done >= r.t_admit >= r.arrival - 1e-9 for r in reqs)
    seen = [rid for _, batch in ex.launched for rid in batch]
    assert sorted(seen) == list(range(400)) and seen == sorted(seen)  # once each, in order
    assert st["arena_peak_bytes"] <= st["arena_bytes"]
    assert st["max_inflight_batches"] >= 2                            # batches overlapped


def test_tiny_budget_forces_queueing():
    ex = FakeExecutor(us_per_product=50.0)
    one = _one(_trace(60, 20000.0))
    eng = serve.Engine(ex, budget_bytes=one, streams=3)
    st = eng.run(_trace(60, 20000.0))
    assert st["completed"] == 60 and st["max_queue"] > 1
    assert st["arena_peak_bytes"] <= one


def test_oversize_rejected_not_queued_forever():
    ex = FakeExecutor()
    tr = _trace(80, 20000.0)
    limit = serve.request_bytes(15, 60) + serve.BATCH_WS_SLACK   # anything larger than N=2^15 x 60 limbs
    eng = serve.Engine(ex, budget_bytes=limit, streams=2)
    st = eng.run(tr)
    big = sum(1 for _, n, L in tr if serve.request_bytes(n, L) + serve.BATCH_WS_SLACK > limit)
    assert big > 0 and st["rejected"] == big and st["completed"] == 80 - big


def test_arena_allocator():
    a = serve.Arena(1 << 20)
    x = a.alloc(1000)
    y = a.alloc(5000)
    z = a.alloc(3000)
    assert x and y and z and a.used == 1024 + 5120 + 3072
    a.release(*y)
    w = a.alloc(4000)
    assert w[0] == y[0]                        # first fit reuses the hole
    a.release(*x)
    a.release(*w)
    a.release(*z)
    assert a.used == 0 and a.free == [(0, 1 << 20)]   # fully coalesced
    assert a.alloc(2 << 20) is None


def test_queue_deadline_times_out_and_frees_nothing_admitted():
    """With a tiny arena the queue backs up; requests waiting longer than the
    deadline leave as timeouts, every other request completes, and the arena
    ends empty."""
    ex = FakeExecutor(us_per_product=400.0)
    tr = _trace(120, 50000.0, seed=3)
    one = _one(tr)
    eng = serve.Engine(ex, budget_bytes=one, streams=2, deadline_s=0.002)
    st = eng.run(tr)
    reqs = st["_requests"]
    assert st["timed_out"] > 0 and st["completed"] + st["timed_out"] == 120
    assert all(r.state in ("done", "timeout") for r in reqs)
    for r in reqs:
        if r.state == "timeout":
            assert r.t_admit is None and r.t_done - r.arrival > 0.002 - 1e-9
    assert eng.arena.used == 0


def test_cancellation():
    """Cancelled while queued or before arrival: dropped; cancelled after
    admission: completes and counts as a late cancellation."""
    ex = FakeExecutor(us_per_product=300.0)
    tr = _trace(100, 40000.0, seed=4)
    one = _one(tr)
    cancels = {5: 0.0, 60: tr[60][0] + 1e-6, 99: 0.0}   # 99 and 5 before they arrive (5 arrives later than 0)
    eng = serve.Engine(ex, budget_bytes=2 * one, streams=2)
    st = eng.run(tr, cancels=cancels)
    reqs = st["_requests"]
    assert reqs[99].state == "cancelled" and reqs[99].t_admit is None
    assert reqs[5].state == "cancelled"
    assert st["cancelled"] + st["completed"] == 100 and st["cancelled"] >= 2
    assert reqs[60].state in ("cancelled", "done")
    assert st["cancelled"] + st["late_cancellations"] <= len(cancels)
    assert eng.arena.used == 0


def test_footprint_counts_operands_output_and_workspace():
    """A request is charged 24 N L bytes (a, b, c) plus its workspace share;
    the arena block of a batch holds the sum, so a budget of exactly one
    request's block admits one such request at a time."""
    assert serve.footprint(16, 10) == 24 * 65536 * 10
    assert serve.request_workspace(16, 10) >= 8 * 65536 * 10        # b's column-pass copy
    assert serve.request_bytes(16, 10) >= serve.footprint(16, 10) + 8 * 65536 * 10
    ex = FakeExecutor(us_per_product=200.0)
    tr = [(0.0, 16, 10), (0.0, 16, 10), (0.0, 16, 10)]
    budget = serve.request_bytes(16, 10) + serve.BATCH_WS_SLACK
    eng = serve.Engine(ex, budget_bytes=budget, streams=3)
    st = eng.run(tr)
    assert st["completed"] == 3 and st["batches"] == 3 and st["max_inflight_batches"] == 1
    assert all(b[1] <= budget for b in ex.blocks) and st["arena_peak_bytes"] <= budget
    # twice the budget: two requests share one block
    eng = serve.Engine(FakeExecutor(us_per_product=200.0), budget_bytes=2 * budget, streams=3)
    st = eng.run(tr)
    assert st["completed"] == 3 and st["mean_batch_requests"] > 1


def test_out_of_order_completion_is_recorded_at_once():
    """A small batch launched after a large one finishes first: its requests
    complete, and its block is freed, while the large batch is still on the
    device (completion is polled for every batch, not just the oldest)."""
    big_end = {}

    def finish_at(batch, now):
        if batch[0].rid == 0:                  # the large request: 50 ms
            big_end["t"] = now + 0.05
            return big_end["t"]
        return now + 0.0005                    # every later batch: 0.5 ms

    ex = FakeExecutor(finish_at=finish_at)
    tr = [(0.0, 17, 60), (0.002, 13, 1), (0.004, 13, 2)]
    eng = serve.Engine(ex, budget_bytes=8 << 30, streams=3)
    st = eng.run(tr)
    reqs = st["_requests"]
    assert st["completed"] == 3 and st["batches"] == 3
    assert reqs[1].t_done < reqs[0].t_done and reqs[2].t_done < reqs[0].t_done
    assert reqs[1].t_done - reqs[1].arrival < 0.02      # not held behind the 50 ms batch
    assert reqs[2].t_done - reqs[2].arrival < 0.02
    assert eng.arena.used == 0
