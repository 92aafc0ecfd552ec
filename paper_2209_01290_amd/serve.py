"""Continuous-batching request loop for negacyclic products.

A request is an RNS product: L limbs of size N (limb l modulo the l-th
largest 60-bit prime q = 1 mod 2N), i.e. L jobs of one pair each. Requests
arrive on a clock (a seeded Poisson trace); the loop

  * queues arrivals in FIFO order;
  * admits requests from the head of the queue while their HBM footprint
    fits the free part of a device arena: 24 N L bytes each (operands a and b,
    output c) plus the batch's workspace (the column-pass copy of b and the
    job table), so requests that arrive while others run are admitted as
    memory frees up;
  * forms a batch of every newly admitted request -- any mix of N -- in one
    arena block, copies each request's operands into its slots there (on
    the batch's stream, ahead of the product), and launches the batch as one
    pm_polymul_jobs call on the next free of S streams (a batch of one
    request as one pm_polymul), so up to S batches overlap on the device;
  * polls the completion event of every batch in flight (batches on
    different streams finish in any order), records each finished request's
    latency (completion seen on the host minus arrival) and frees its block.

Operand sources stay resident on the device: per N, a pool of operand sets
(60 limbs each) drawn once with the device generator; request r's operands
are copied from pool entry r mod pool_size (this copy stands for the request
bringing its operands). Twiddle tables for every (N, limb) are resident.

The scheduling logic is independent of the device: `Engine` drives an
executor object; `GpuExecutor` runs the library, tests on the CPU use a fake.

Usage:  python -m paper_2209_01290_amd.serve --rates 2000,5000,10000,20000,50000
"""
from __future__ import annotations

import argparse
import collections
import ctypes
import gc
import json
import time

import numpy as np

from . import workloads

SEED = 220901290 + 5
ALIGN = 256

# pm_job as a numpy record (layout of include/pm.h: two uint32, one uint64, five pointers)
JOB_DTYPE = np.dtype([("log2n", "<u4"), ("count", "<u4"), ("q", "<u8"), ("psi_br", "<u8"),
                      ("psi_inv_br", "<u8"), ("a", "<u8"), ("b", "<u8"), ("c", "<u8")])


class Arena:
    """First-fit allocator of byte ranges of one device buffer (host-side book-keeping)."""

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)]          # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, n: int):
        n = (n + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off, n
        return None

    def largest_free(self) -> int:
        return max((ln for _, ln in self.free), default=0)

    def release(self, off: int, n: int):
        self.used -= n
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, (off, n))
        # coalesce with neighbours
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            self.free[i] = (off, n + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)


class Request:
    __slots__ = ("rid", "arrival", "log2n", "limbs", "t_admit", "t_done", "slot", "state")

    def __init__(self, rid, arrival, log2n, limbs):
        self.rid, self.arrival, self.log2n, self.limbs = rid, arrival, log2n, limbs
        self.t_admit = self.t_done = None
        self.slot = None                # arena byte offset of its operand a (then b, then c)
        self.state = "pending"


def _align(n: int) -> int:
    return (n + ALIGN - 1) // ALIGN * ALIGN


def footprint(log2n: int, limbs: int) -> int:
    """HBM bytes of a request's words: operands a and b and output c, 24 N L."""
    return 24 * (1 << log2n) * limbs


def request_workspace(log2n: int, limbs: int) -> int:
    """Upper bound of the workspace bytes a request adds to its batch: the
    column-pass copy of b when the product runs in two passes, plus its
    job-table entries (one record of at most 256 bytes and at most 80
    work-item slots of 4 bytes per limb)."""
    N = 1 << log2n
    return (N * limbs * 8 if log2n > 12 else 0) + limbs * 576


def request_bytes(log2n: int, limbs: int) -> int:
    """Arena bytes a request takes in its batch's block: its footprint and its
    share of the batch workspace, each 256-byte aligned."""
    return _align(footprint(log2n, limbs)) + _align(request_workspace(log2n, limbs))


BATCH_WS_SLACK = 8192     # per batch: alignment of the workspace parts


class Engine:
    """deadline_s: a request still waiting in the queue that long after its
    arrival is dropped (state "timeout"); admitted requests always complete.
    run(cancels=...) takes {request id: time}: a request still queued at that
    time is dropped (state "cancelled"); a request already admitted or on the
    device completes and is counted as a late cancellation."""

    def __init__(self, executor, budget_bytes: int, streams: int = 3, max_batch_products: int = 4096,
                 deadline_s: float | None = None):
        self.ex = executor
        self.arena = Arena(budget_bytes)
        self.streams = streams
        self.max_batch_products = max_batch_products
        self.deadline_s = deadline_s

    def run(self, trace, time_scale: float = 1.0, on_complete=None, cancels=None):
        """trace: [(arrival_s, log2n, limbs)] sorted by arrival. Returns stats.
        The garbage collector is held off while the loop runs (its pauses
        would show up as request latency)."""
        gc_was = gc.isenabled()
        gc.disable()
        try:
            return self._run(trace, time_scale, on_complete, cancels or {})
        finally:
            if gc_was:
                gc.enable()

    def _run(self, trace, time_scale, on_complete, cancels):
        reqs = [Request(i, t * time_scale, n, L) for i, (t, n, L) in enumerate(trace)]
        queue = collections.deque()
        inflight = []                           # (handle, [requests], arena block)
        max_inflight = 0
        rejected = []                           # rejected at arrival, timed out or cancelled
        late_cancel = 0
        cancel_at = sorted((t * time_scale, rid) for rid, t in cancels.items())
        drop_now, drop_on_arrival = set(), set()
        ci = 0
        nxt = 0
        done = 0
        batches, batch_sizes, max_queue = 0, [], 0
        t0 = time.monotonic()
        while done + len(rejected) < len(reqs):
            now = time.monotonic() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                if r.rid in drop_on_arrival:
                    drop_on_arrival.discard(r.rid)
                    r.state = "cancelled"
                    r.t_done = now
                    rejected.append(r)
                elif request_bytes(r.log2n, r.limbs) + BATCH_WS_SLACK > self.arena.size:
                    r.state = "rejected"
                    rejected.append(r)
                else:
                    queue.append(r)
                nxt += 1
            # cancellations due by now: queued requests leave the queue, ones
            # not yet arrived are dropped on arrival, admitted ones complete
            while ci < len(cancel_at) and cancel_at[ci][0] <= now:
                r = reqs[cancel_at[ci][1]]
                if r.state == "pending":
                    (drop_now if r.rid < nxt else drop_on_arrival).add(r.rid)
                elif r.state == "admitted":
                    late_cancel += 1
                ci += 1
            expired = self.deadline_s is not None and queue and now - queue[0].arrival > self.deadline_s
            if expired or drop_now:
                kept = collections.deque()
                for r in queue:
                    if r.rid in drop_now:
                        r.state = "cancelled"
                    elif self.deadline_s is not None and now - r.arrival > self.deadline_s:
                        r.state = "timeout"
                    else:
                        kept.append(r)
                        continue
                    r.t_done = now
                    rejected.append(r)
                queue = kept
                drop_now.clear()
            max_queue = max(max_queue, len(queue))
            # completions: every batch in flight is polled, so a batch that
            # finishes before an earlier one is recorded and freed at once
            if inflight:
                still = []
                for ent in inflight:
                    handle, batch, block = ent
                    if not self.ex.done(handle):
                        still.append(ent)
                        continue
                    tdone = time.monotonic() - t0
                    for r in batch:
                        r.t_done = tdone
                        r.state = "done"
                        if on_complete is not None:
                            on_complete(r, self.ex)
                        done += 1
                    self.arena.release(*block)
                    self.ex.finish(handle)
                inflight = still
            # admission and launch: requests from the head of the queue while
            # the batch's block (footprints and workspace) fits the arena
            if queue and len(inflight) < self.streams:
                batch, products, need = [], 0, BATCH_WS_SLACK
                room = self.arena.largest_free()
                while queue and products + queue[0].limbs <= self.max_batch_products:
                    r = queue[0]
                    add = request_bytes(r.log2n, r.limbs)
                    if need + add > room:
                        break
                    queue.popleft()
                    r.t_admit, r.state = now, "admitted"
                    batch.append(r)
                    products += r.limbs
                    need += add
                if batch:
                    block = self.arena.alloc(need)
                    assert block is not None, "arena block smaller than its largest free extent"
                    handle = self.ex.launch(batch, batches, block)
                    inflight.append((handle, batch, block))
                    max_inflight = max(max_inflight, len(inflight))
                    batches += 1
                    batch_sizes.append(len(batch))
                    continue
            if not inflight and not queue and nxt < len(reqs):
                dt = reqs[nxt].arrival - (time.monotonic() - t0)
                if dt > 0:
                    time.sleep(min(dt, 0.002))
            elif inflight:
                time.sleep(0)   # yield; completion is polled
        wall = time.monotonic() - t0
        ok = [r for r in reqs if r.state == "done"]
        lat = np.array([r.t_done - r.arrival for r in ok]) * 1e3
        n16 = sum(((1 << r.log2n) * r.log2n * r.limbs) for r in ok) / float((1 << 16) * 16)
        span = (max(r.t_done for r in ok) - min(r.arrival for r in ok)) if ok else 0.0
        return {
            "requests": len(reqs), "completed": len(ok),
            "rejected": sum(1 for r in rejected if r.state == "rejected"),
            "timed_out": sum(1 for r in rejected if r.state == "timeout"),
            "cancelled": sum(1 for r in rejected if r.state == "cancelled"),
            "late_cancellations": late_cancel,
            "limb_products": int(sum(r.limbs for r in ok)),
            "wall_s": round(wall, 4),
            "throughput_req_s": round(len(ok) / span, 1) if span > 0 else None,
            "throughput_polymul_s": round(sum(r.limbs for r in ok) / span, 1) if span > 0 else None,
            "throughput_n16_equiv_s": round(n16 / span, 1) if span > 0 else None,
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
                           "p99": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
                           "mean": round(float(lat.mean()), 3) if len(lat) else None},
            "batches": batches, "mean_batch_requests": round(float(np.mean(batch_sizes)), 2) if batch_sizes else 0,
            "max_queue": max_queue, "max_inflight_batches": max_inflight,
            "arena_peak_bytes": self.arena.peak, "arena_bytes": self.arena.size,
            "_requests": reqs,
        }


class GpuExecutor:
    """Runs batches with pm_polymul_jobs in blocks of one device arena, with
    operand pools and tables resident. In a batch's block each request has
    three [limbs][N] slots (a, b, c) and the batch's workspace follows them;
    the request's operands are copied into its slots on the batch's stream
    before the product. A batch of one request (the common case below
    saturation) runs as one pm_polymul over its limbs instead
    (single_request_path): its slots and tables are contiguous [limbs][N]
    blocks, and pm_polymul takes the tuned small-batch plan when the request
    is small enough to be latency-bound. Each batch runs on a stream that no
    batch in flight is using."""

    def __init__(self, budget_bytes: int, streams: int = 3, pool: int = 4, max_limbs: int = 60,
                 log2ns=workloads.SERVE_LOG2N, device="cuda", seed: int = SEED,
                 single_request_path: bool = True):
        import torch
        from . import lib, synth
        self.torch, self.lib = torch, lib
        lib.load()
        self.dev = torch.device(device)
        self.arena_t = torch.empty(budget_bytes // 8, dtype=torch.int64, device=self.dev)
        self.base = self.arena_t.data_ptr()
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(streams)]
        self.busy = [False] * streams
        self.pool = pool
        self.max_limbs = max_limbs
        self.tables = workloads.Tables(self.dev)
        self.inputs = {}
        self.seed = seed
        for log2n in log2ns:
            N = 1 << log2n
            prm = self.tables.get(log2n, max_limbs)
            a = torch.empty((pool, max_limbs, N), dtype=torch.int64, device=self.dev)
            b = torch.empty_like(a)
            for p in range(pool):
                synth.uniform_mod_device([synth.key(seed, p, l, 0, 0) for l in range(max_limbs)], N,
                                         prm.q[:max_limbs], a[p])
                synth.uniform_mod_device([synth.key(seed, p, l, 0, 1) for l in range(max_limbs)], N,
                                         prm.q[:max_limbs], b[p])
            self.inputs[log2n] = (a, b)
        # job records per N for all max_limbs limbs (moduli and tables),
        # operand and output pointers aside: a request takes the first L rows
        self.rows, self.l_off = {}, {}
        for log2n in log2ns:
            N = 1 << log2n
            prm = self.tables.get(log2n, max_limbs)
            lidx = np.arange(max_limbs, dtype=np.uint64) * np.uint64(N * 8)
            self.l_off[log2n] = lidx
            rows = np.zeros(max_limbs, dtype=JOB_DTYPE)
            rows["log2n"] = log2n
            rows["count"] = 1
            rows["q"] = np.array(prm.q[:max_limbs], dtype=np.uint64)
            rows["psi_br"] = np.uint64(prm.psi_br.data_ptr()) + lidx
            rows["psi_inv_br"] = np.uint64(prm.psi_inv_br.data_ptr()) + lidx
            self.rows[log2n] = rows
        self.single_request_path = single_request_path
        self.qarr = {n: (ctypes.c_uint64 * max_limbs)(*self.tables.get(n, max_limbs).q[:max_limbs])
                     for n in log2ns}
        torch.cuda.synchronize()

    def budget(self):
        return self.arena_t.numel() * 8

    def resident_bytes(self):
        t = sum(2 * x[0].numel() * 8 for x in self.inputs.values())
        t += sum(2 * p.psi_br.numel() * 8 for p in self.tables.by_n.values())
        return t + self.budget()

    def job_rows(self, r, a_ptr, b_ptr, c_ptr):
        """pm_job records of request r with its operands and output at the given addresses."""
        rows = self.rows[r.log2n][:r.limbs].copy()
        off = self.l_off[r.log2n][:r.limbs]
        rows["a"] = np.uint64(a_ptr) + off
        rows["b"] = np.uint64(b_ptr) + off
        rows["c"] = np.uint64(c_ptr) + off
        return rows

    def pool_operands(self, r):
        """(a, b) of request r in its operand pool entry: [limbs, N] views."""
        a, b = self.inputs[r.log2n]
        p = r.rid % self.pool
        return a[p, :r.limbs], b[p, :r.limbs]

    def _slot(self, byte_off, r):
        N = 1 << r.log2n
        w = byte_off // 8
        return self.arena_t[w: w + r.limbs * N].view(r.limbs, N)

    def slots(self, r):
        """The device views (a, b, c) of request r's slots in its batch's block."""
        nb = 8 * (1 << r.log2n) * r.limbs
        return self._slot(r.slot, r), self._slot(r.slot + nb, r), self._slot(r.slot + 2 * nb, r)

    def output(self, r):
        return self.slots(r)[2]

    def launch(self, batch, k, block):
        i = self.busy.index(False)          # the engine keeps at most len(streams) batches in flight
        self.busy[i] = True
        s = self.streams[i]
        off = block[0]
        for r in batch:
            r.slot = off
            off += _align(footprint(r.log2n, r.limbs))
        ws_off = _align(off)
        ws_bytes = block[0] + block[1] - ws_off
        with self.torch.cuda.stream(s):
            for r in batch:
                a_src, b_src = self.pool_operands(r)
                a_dst, b_dst, _ = self.slots(r)
                a_dst.copy_(a_src, non_blocking=True)
                b_dst.copy_(b_src, non_blocking=True)
        if len(batch) == 1 and self.single_request_path:
            r = batch[0]
            a, b, c = self.slots(r)
            prm = self.tables.get(r.log2n, self.max_limbs)
            self.lib.pm_polymul_raw(a.data_ptr(), b.data_ptr(), c.data_ptr(), 1 << r.log2n, r.limbs, 1,
                                    self.qarr[r.log2n], prm.psi_br.data_ptr(), prm.psi_inv_br.data_ptr(),
                                    self.base + ws_off, s.cuda_stream)
        else:
            jobs = np.concatenate([self.job_rows(r, *(t.data_ptr() for t in self.slots(r))) for r in batch])
            self.lib.pm_polymul_jobs_raw(jobs.ctypes.data, len(jobs), self.base + ws_off, ws_bytes, s.cuda_stream)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return (ev, i)

    def run_alone(self, r):
        """Request r on its own through pm_polymul_jobs, reading its operands
        in the pool, into a fresh output tensor."""
        torch = self.torch
        out = torch.empty((r.limbs, 1 << r.log2n), dtype=torch.int64, device=self.dev)
        a, b = self.pool_operands(r)
        jobs = self.job_rows(r, a.data_ptr(), b.data_ptr(), out.data_ptr())
        need = self.lib.pm_polymul_jobs_workspace_bytes_raw(jobs.ctypes.data, len(jobs))
        ws = torch.empty(max(need // 8 + 64, 64), dtype=torch.int64, device=self.dev)
        self.lib.pm_polymul_jobs_raw(jobs.ctypes.data, len(jobs), ws.data_ptr(), ws.numel() * 8,
                                     torch.cuda.current_stream(self.dev).cuda_stream)
        torch.cuda.synchronize()
        return out

    def done(self, handle):
        return handle[0].query()

    def finish(self, handle):
        self.busy[handle[1]] = False


def warm_up(ex):
    """One request per size through the batched entry point before any timing:
    the first launch of each kernel loads its code, which would otherwise land
    in the first requests' latency."""
    for i, log2n in enumerate(workloads.SERVE_LOG2N):
        ex.run_alone(Request(i, 0.0, log2n, 2))


def run_rates(rates, nreq, budget_gib=32.0, streams=3, seed=SEED, verbose=True, ex=None,
              max_batch_products=4096):
    ex = ex or GpuExecutor(int(budget_gib * (1 << 30)), streams=streams, seed=seed)
    warm_up(ex)
    out = []
    for rate in rates:
        trace = [(t, n, L) for (t, n, L) in workloads.serving_requests(seed + int(rate), nreq, rate)]
        eng = Engine(ex, ex.budget(), streams=streams, max_batch_products=max_batch_products)
        st = eng.run(trace)
        st.pop("_requests")
        st["offered_rate_req_s"] = rate
        out.append(st)
        if verbose:
            print(json.dumps(st), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="2000,5000,10000,20000,50000")
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--streams", type=int, default=3)
    ap.add_argument("--max-batch-products", type=int, default=4096, help="limb-products per batch at most")
    a = ap.parse_args()
    from . import lib
    lib.load()
    lib.apply_tune_db()
    run_rates([float(x) for x in a.rates.split(",")], a.requests, a.budget_gib, a.streams,
              max_batch_products=a.max_batch_products)


if __name__ == "__main__":
    main()
