#!/usr/bin/env python3
"""Throughput benchmark: exact negacyclic polymul/s at N = 2^16 on one MI355X.

Workload (one step): 48 RNS limbs, each with its own 60-bit prime
q = 1 mod 2^17 (the 48 largest below 2^60), 8 independent polynomial pairs
per limb, i.e. 384 products c = a (*) b in Z_q[x]/(x^65536 + 1), operands
uniform in [0, q) from the seeded SplitMix64 generator. A step is one call of
the batched entry point pm_polymul over the whole batch: forward merged CT
NTT of a and b, pointwise product, halved merged GS inverse (software-
pipelined over two chunks of 24 limbs: 4 launches). Inputs, twiddle tables
and outputs stay resident in HBM; the timed region holds only kernels.

Reported beside the batched throughput:
  plain       the same 384 products as 384 separate pm_polymul calls (one
              launch sequence per product, no batching across products)
  stagewise   pm_polymul_stagewise (one launch per NTT stage) on the batch
  ntt_fwd     standalone forward transforms of the 384 a operands
  roofline    the dominant kernel's live average duration (HIP events on its
              own stream) against the VALU issue ceiling, with the HBM view
  three_pass  the same step without pipelining (column, row, column pass)
              and the row pass's own roofline
  cpu_baseline  the CPU oracle on a bounded sample of the same products

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_LOG2, LIMBS, POLYS = 16, 48, 8
SEED = 220901290 + 3

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one 32-bit VALU lane-op per
# lane per cycle; HBM3E peak 8 TB/s.
CLOCK_MHZ = 2400.0
PEAK_VALU_TOPS = 256 * 4 * 16 * CLOCK_MHZ * 1e6 / 1e12
PEAK_HBM_GBPS = 8000.0
# VALU instructions per unit of the method's work, counted in the ISA of
# register-resident loops over the device arithmetic (modarith.hpp). A GS
# butterfly takes its twiddle halved (38 instructions) and each twiddle is
# halved once for the butterflies that share it (6 instructions; 15 twiddles
# per 32 butterflies in the radix-16 rounds).
TW_PER_GS = 15 / 32
OPS_CT, OPS_GS, OPS_MUL = 32, 38 + 6 * TW_PER_GS, 22


# The same counts by instruction class: each class is priced by the probe
# instruction that stands for it (pm_probe_valu's measured issue rates), which
# gives the VALU-bound time of a launch for this instruction mix.
MIX = {
    "ct": {"v_mad_u64_u32": 8, "v_mul_hi_u32": 1, "v_mul_lo_u32": 2, "v_add3_u32": 1, "v_alignbit_b32": 2,
           "v_lshl_add_u64": 2, "v_sub_co_u32": 15, "v_mov_b32": 1},
    "gs": {"v_mad_u64_u32": 8, "v_mul_hi_u32": 1, "v_mul_lo_u32": 2, "v_add3_u32": 2 + TW_PER_GS,
           "v_alignbit_b32": 2, "v_lshl_add_u64": 4 + 2 * TW_PER_GS, "v_sub_co_u32": 15,
           "v_xor_b32": 3 + 3 * TW_PER_GS, "v_mov_b32": 1},
    "mul": {"v_mad_u64_u32": 8, "v_mul_hi_u32": 1, "v_mul_lo_u32": 2, "v_add3_u32": 1, "v_alignbit_b32": 2,
            "v_sub_co_u32": 7, "v_mov_b32": 1},
}
assert all(abs(sum(MIX[u].values()) - o) < 1e-9 for u, o in (("ct", OPS_CT), ("gs", OPS_GS), ("mul", OPS_MUL)))

# The same counts for 32-bit words (modarith32.hpp), moduli with m <= 29 /
# m = 30 (one more shift per modular product).
OPS32 = {29: (14, 17 + 4 * TW_PER_GS, 7), 30: (15, 18 + 4 * TW_PER_GS, 8)}


def alg_ops(name: str, N: int, limbs: int, polys: int, ops=(OPS_CT, OPS_GS, OPS_MUL),
            launches_per_step: int = 1) -> float:
    """Algorithmic VALU lane-ops one launch of kernel `name` performs
    (row_* / row32_*: fused row pass; col_* / col32_*: column pass; pipe_*:
    the software-pipelined product, whose launches_per_step launches share the
    row and column work of one batch)."""
    ct, gs, mul = ops
    kind, _, rest = name.partition("_")
    if kind in ("row", "row32"):
        mode, logc = rest.split("_c")
        C = 1 << int(logc)
        rows = limbs * polys * (N // C)
        half = (C // 2) * int(logc)            # butterflies of one row transform
        if mode == "mul":
            per = 2 * half * ct + C * mul + half * gs
        elif mode == "fwd":
            per = half * ct
        elif mode == "inv":
            per = half * gs
        else:
            return float("nan")
        return float(rows * per)
    if kind in ("col", "col32"):
        mode, logr = rest.split("_r")
        R = 1 << int(logr)
        cols = (N // R) * limbs * polys
        nops = 2 if mode == "fwd" else 1
        per = (R // 2) * int(logr) * (ct if mode == "fwd" else gs)
        return float(cols * nops * per)
    if kind == "pipe":
        mode, logc = rest.split("_c")
        if mode != "mul":
            return float("nan")
        logr = N.bit_length() - 1 - int(logc)
        step = sum(alg_ops(k, N, limbs, polys, ops) for k in
                   ("row_mul_c%s" % logc, "col_fwd_r%d" % logr, "col_inv_r%d" % logr))
        return step / launches_per_step
    return float("nan")


def mix_ceiling(name: str, N: int, limbs: int, polys: int, rates: dict) -> float:
    """T lane-ops/s a launch of `name` could reach if the VALU issued every
    instruction of its mix at the rate pm_probe_valu measured for its class."""
    secs = alg_ops(name, N, limbs, polys,
                   ops=tuple(sum(n / rates[i] for i, n in MIX[u].items()) for u in ("ct", "gs", "mul")))
    return alg_ops(name, N, limbs, polys) / secs / 1e12


# The sources the reported kernels are compiled from: the counter summary
# stays valid while these are unchanged (host-only files do not matter).
ROW_KERNEL_SOURCES = ("modarith.hpp", "modarith32.hpp", "ntt_device.hpp", "ntt_row.hpp", "pm_internal.hpp",
                      "row_kernel.inc", "row_12.hip", "row_fixed.inc", "row_12r.hip", "pm_kernels.hip",
                      "pipe_kernels.hip", "pm_pipe.hpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_01290_amd", "csrc")
    for f in ROW_KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else float(k["hbm_bytes_per_launch"])


def pct(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def host_cpus():
    """CPUs this process may run on (its affinity mask, capped by the job's
    OMP_NUM_THREADS share where one is set), the machine's CPU count and model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(avail, int(share)) if share.isdigit() and int(share) > 0 else avail
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": max(1, threads), "affinity_cpus": avail, "nproc": os.cpu_count(),
            "omp_num_threads": share or None, "cpu_model": model}


def cpu_baseline(N, qs, a_host, b_host, gpu_c, run_s=2.5, runs=5):
    """The oracle (plain C, % reductions) on a bounded sample of the same
    products: one product per thread over every CPU the job may use, `runs`
    runs of about `run_s` seconds, median; and the same on one core. Checks
    the GPU's outputs for the sampled pairs on the way."""
    import oracle
    o = oracle.default()
    cpus = host_cpus()
    threads = cpus["threads"]
    pairs = [(i % len(qs), (i // len(qs)) % a_host.shape[1]) for i in range(threads)]
    tables = {}
    for l, _ in pairs:
        if l not in tables:
            tables[l] = o.psi_tables(qs[l], N)
    t0 = time.perf_counter()
    l0, p0 = pairs[0]
    c0 = o.polymul_ntt(a_host[l0, p0], b_host[l0, p0], qs[l0], *tables[l0])
    t1 = time.perf_counter() - t0
    if not np.array_equal(c0, gpu_c[l0, p0]):
        raise SystemExit("GPU output differs from the oracle on limb %d pair %d" % (l0, p0))

    def timed_run(nthreads, reps):
        def work(k):
            l, p = pairs[k]
            for _ in range(reps):
                c = o.polymul_ntt(a_host[l, p], b_host[l, p], qs[l], *tables[l])
            return k, c
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(nthreads) as ex:
            outs = list(ex.map(work, range(nthreads)))
        wall = time.perf_counter() - t0
        for k, c in outs:
            l, p = pairs[k]
            if not np.array_equal(c, gpu_c[l, p]):
                raise SystemExit("GPU output differs from the oracle on limb %d pair %d" % (l, p))
        return nthreads * reps / wall

    reps = max(1, int(run_s / max(t1, 1e-6) / 1.3))
    rates = [timed_run(threads, reps) for _ in range(runs)]
    reps1 = max(1, int(0.5 / max(t1, 1e-6)))
    rates1 = [timed_run(1, reps1) for _ in range(runs)]
    # context for the one-product case: the O(N^2) schoolbook and the NTT
    # route of the oracle for one N = 1024 product, one thread
    from paper_2209_01290_amd import synth
    q1 = 2 ** 60 - 2 ** 14 + 1
    a1, b1 = synth.operands(220901290 + 1, [q1], 1, 1024)
    t0 = time.perf_counter()
    s1 = o.polymul_schoolbook(a1[0, 0], b1[0, 0], q1)
    t_school = time.perf_counter() - t0
    f1, i1 = o.psi_tables(q1, 1024)
    t0 = time.perf_counter()
    n1 = o.polymul_ntt(a1[0, 0], b1[0, 0], q1, f1, i1)
    t_ntt = time.perf_counter() - t0
    if not np.array_equal(s1, n1):
        raise SystemExit("oracle schoolbook and NTT products differ at N=1024")
    return {"value": round(pct(rates, 50), 1), "unit": "polymul/s", "cores": threads, "kind": "oracle",
            "sample": "N=2^16 products of the benchmark workload (limbs %s), %d per thread per run, "
                      "%d threads, median of %d runs; oracle transforms with %% reductions, gcc -O2"
                      % (sorted(set(l for l, _ in pairs)), reps, threads, runs),
            "runs_polymul_s": [round(r, 1) for r in rates],
            "single_core": {"value": round(pct(rates1, 50), 1), "unit": "polymul/s",
                            "runs_polymul_s": [round(r, 1) for r in rates1], "products_per_run": reps1},
            "host": cpus,
            "n1024_one_product_us": {"schoolbook": round(t_school * 1e6, 1), "ntt": round(t_ntt * 1e6, 1),
                                     "threads": 1}}


def mixed_batch(torch, lib, dev, launches=5):
    """The batched mixed workload: 512 requests, N uniform on 2^12..2^17, 1..48
    limbs, all in one plan (one graph launch). Its default job table is the
    software-pipelined one; the same batch as a three-pass table (one launch
    per pass of Eq. 2) is timed in alternating blocks, and one pm_polymul call
    per request (same kernels, batched across limbs only) beside both."""
    from paper_2209_01290_amd import workloads
    reqs = workloads.mixed_requests(220901290 + 4)
    mb = workloads.MixedBatch(reqs, 220901290 + 4, dev)
    work16 = sum((1 << n) * n for n, L in reqs for _ in range(L)) / float((1 << 16) * 16)
    stream = torch.cuda.current_stream(dev)
    plans = {}
    try:
        for name, chunks in (("pipelined", -1), ("three_pass", 0)):
            lib.pm_tune_set_jobs_pipeline(chunks)
            plans[name] = lib.pm_plan_create(mb.jobs)
        lib.pm_tune_set_jobs_pipeline(-1)
        per = {k: [] for k in plans}
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(launches + 1)]
        for _rep in range(2):
            for name, plan in plans.items():
                for _ in range(2):
                    lib.pm_plan_launch(plan)
                torch.cuda.synchronize()
                ev[0].record(stream)
                for k in range(launches):
                    lib.pm_plan_launch(plan)
                    ev[k + 1].record(stream)
                torch.cuda.synchronize()
                per[name] += [ev[k].elapsed_time(ev[k + 1]) for k in range(launches)]
        dev_bytes = lib.pm_plan_device_bytes(plans["pipelined"])
        # the pipelined plan's kernels, timed one by one (graph launch off:
        # the same launches issued directly, each bracketed by events)
        lib.pm_tune_set_jobs_pipeline(-1)
        direct = lib.pm_plan_create(mb.jobs, 1)
        try:
            lib.pm_plan_launch(direct)
            torch.cuda.synchronize()
            lib.pm_prof_read(reset=True)
            lib.pm_prof_enable(True)
            for _ in range(2):
                lib.pm_plan_launch(direct)
            torch.cuda.synchronize()
            lib.pm_prof_enable(False)
            kern = lib.pm_prof_read(reset=True)
        finally:
            lib.pm_plan_destroy(direct)
    finally:
        lib.pm_tune_set_jobs_pipeline(-1)
        for plan in plans.values():
            lib.pm_plan_destroy(plan)
    ms = pct(per["pipelined"], 50)
    ms3 = pct(per["three_pass"], 50)
    maxws = max(lib.pm_polymul_workspace_bytes(1 << n, L, 1) for n, L in reqs)
    ws = torch.empty(max(maxws // 8, 1), dtype=torch.int64, device=dev)

    def per_request():
        for r, (n, L) in enumerate(reqs):
            prm = mb.tables.get(n, 0)
            a, b, c = mb.request_limbs(r)
            lib.pm_polymul(a, b, c, 1 << n, L, 1, prm.q[:L], prm.psi_br[:L], prm.psi_inv_br[:L], ws)

    per_request()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    per_request()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    # algorithmic VALU work of the batch (the per-unit counts of the uniform
    # step): butterflies of the three transforms and the pointwise products
    ops = sum(L * (1 << n) * (n * (OPS_CT + OPS_GS / 2.0) + OPS_MUL) for n, L in reqs)
    pipe_ms = sum(v[1] for k, v in kern.items() if k == "jobs_pipe_mul_c12") / 2.0
    return {"what": "512 requests, N uniform on 2^12..2^17, 1..48 limbs (%d limb-products), one plan "
                    "(HIP graph) launch per batch" % mb.products,
            "products": mb.products, "ms_per_batch": round(ms, 3), "p99_ms": round(pct(per["pipelined"], 99), 3),
            "timing": "median of 2 alternating blocks of %d launches per form" % launches,
            "value": round(mb.products / ms * 1e3, 1), "unit": "polymul/s",
            "n16_equivalent_per_s": round(work16 / ms * 1e3, 1),
            "jobs_pipeline_chunks": lib.pm_tune_get_jobs_pipeline(),
            "pipelined_launches": {k: v[0] // 2 for k, v in kern.items()},
            "kernels_ms_per_batch": {k: round(v[1] / 2.0, 4) for k, v in sorted(kern.items())},
            "valu": {"alg_ops_per_batch": ops, "achieved_T_step": round(ops / (ms / 1e3) / 1e12, 3),
                     "achieved_T_pipe_kernels": round(ops / (pipe_ms / 1e3) / 1e12, 3) if pipe_ms else None,
                     "peak_T": round(PEAK_VALU_TOPS, 3)},
            "three_pass": {"ms_per_batch": round(ms3, 3), "n16_equivalent_per_s": round(work16 / ms3 * 1e3, 1),
                           "pipelined_over_three_pass": round(ms3 / ms, 4)},
            "plan_device_bytes": dev_bytes,
            "per_request_ms": round(ms_plain, 3),
            "per_request_value": round(mb.products / ms_plain * 1e3, 1),
            "batched_over_per_request": round(ms_plain / ms, 3)}


def config2(torch, lib, dev, steps=20):
    """The paper's global-memory baseline shape: N = 2^14, 32 limbs (the 32
    largest 60-bit primes q = 1 mod 2^15), one pair per limb, through the plain
    per-stage path pm_polymul_stagewise (14 forward stage launches over a and
    b, one pointwise launch, 14 halved inverse stage launches; each launch
    covers all limbs), with the batched pm_polymul beside it. Per-pass HBM
    rate from the library's event timer: algorithmic bytes per launch (the
    words each launch reads and writes once) over its average duration."""
    from paper_2209_01290_amd import synth
    N, L, P = 1 << 14, 32, 1
    prm = lib.Params(N, L, device=dev)
    a, b = synth.operands(220901290 + 2, prm.q, P, N)
    da, db = lib.to_device(a, dev), lib.to_device(b, dev)
    dc = torch.empty_like(da)
    sws = torch.empty(max(lib.pm_polymul_stagewise_workspace_bytes(N, L, P) // 8, 1), dtype=torch.int64,
                      device=dev)
    bws = torch.empty(max(lib.pm_polymul_workspace_bytes(N, L, P) // 8, 1), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    plain = lambda: lib.pm_polymul_stagewise(da, db, dc, N, L, P, prm.q, prm.psi_br, prm.psi_inv_br, sws)
    batched = lambda: lib.pm_polymul(da, db, dc, N, L, P, prm.q, prm.psi_br, prm.psi_inv_br, bws)

    def per_step(fn):
        for _ in range(5):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]

    t_plain, t_batched = per_step(plain), per_step(batched)
    lib.pm_prof_read(reset=True)
    lib.pm_prof_enable(True)
    for _ in range(steps):
        plain()
    torch.cuda.synchronize()
    lib.pm_prof_enable(False)
    kern = lib.pm_prof_read(reset=True)
    words = L * P * N
    # bytes each launch moves once: a stage reads and writes its operands
    # (a and b forward, c inverse) and reads its limbs' twiddles; pointwise
    # reads two operands and writes one (the plain path moves every word
    # 2 x 29 times per step: no stage fusion)
    tw = L * (N - 1) // 14 * 8          # twiddle words per stage launch, on average over the 14 stages
    alg_bytes = {"stage_fwd": 2 * 2 * words * 8 + tw, "stage_inv": 2 * words * 8 + tw, "pointwise": 3 * words * 8}
    passes = {}
    for name, (n, ms) in sorted(kern.items()):
        avg = ms / n
        passes[name] = {"launches_per_step": n // steps, "avg_ms": round(avg, 5),
                        "alg_bytes": alg_bytes.get(name),
                        "GBps": round(alg_bytes[name] / (avg / 1e3) / 1e9, 1) if name in alg_bytes else None}
    ms_plain, ms_b = sum(t_plain) / steps, sum(t_batched) / steps
    b_alg = L * P * 24 * N + L * 16 * N
    return {"what": "N=2^14, 32 limbs x 1 pair, 60-bit primes; pm_polymul_stagewise: one launch per stage "
                    "(29 launches per step), each over all limbs",
            "value": round(L * P / ms_plain * 1e3, 1), "unit": "polymul/s", "ms_per_step": round(ms_plain, 4),
            "latency_ms": {"p50": round(pct(t_plain, 50), 4), "p99": round(pct(t_plain, 99), 4)},
            "per_pass": passes,
            "hbm_roofline": {"alg_bytes_per_step": b_alg,
                             "frac": round(b_alg / (ms_plain / 1e3) / 1e9 / PEAK_HBM_GBPS, 4)},
            "batched": {"value": round(L * P / ms_b * 1e3, 1), "unit": "polymul/s", "ms_per_step": round(ms_b, 4),
                        "latency_ms": {"p50": round(pct(t_batched, 50), 4), "p99": round(pct(t_batched, 99), 4)},
                        "what": "pm_polymul on the same batch (tuned plan)"},
            "batched_over_plain": round(ms_plain / ms_b, 3)}


def alternate(torch, stream, fns, blocks=4, per=10):
    """Median ms per call of each function in `fns` ({name: fn}), timed in
    alternating blocks of `per` calls (each block after 2 untimed calls), so
    that clock and thermal drift fall on every variant alike."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = {k: [] for k in fns}
    for _ in range(blocks):
        for k, fn in fns.items():
            for _ in range(2):
                fn()
            e0.record(stream)
            for _ in range(per):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t[k].append(e0.elapsed_time(e1) / per)
    return {k: pct(v, 50) for k, v in t.items()}


def _median_call_us(torch, stream, fn, reps):
    """Median device time of one call over `reps` back-to-back calls (events
    between consecutive calls on the same stream)."""
    for _ in range(5):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(reps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    return pct([ev[k].elapsed_time(ev[k + 1]) * 1e3 for k in range(reps)], 50)


def _graph_call_us(torch, fn, calls=20, reps=10):
    """Device time of one call without host overhead: `calls` consecutive calls
    captured in one HIP graph, the graph replayed `reps` times; median per call."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(calls):
            fn()
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for k in range(reps):
        g.replay()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) * 1e3 / calls for k in range(reps))
    del g
    return per[len(per) // 2]


def words32(torch, lib, dev, steps=20):
    """The 32-bit word path (moduli up to 30 bits, Alg. 4 with beta = 32):
    single-transform latency at N = 2^14 and 2^16 beside 62-bit moduli on
    64-bit words (the rows of the paper's comparison table in Sec. VII; device
    time per call from HIP-graph replays, and the time per call when each is
    launched from Python), and the workload-size
    trade-off: the 2880-bit modulus of the headline workload as 96 30-bit
    limbs on 32-bit words against 48 60-bit limbs on 64-bit words."""
    from paper_2209_01290_amd import synth
    stream = torch.cuda.current_stream(dev)
    lat = []
    for log2n in (14, 16):
        N = 1 << log2n
        for bits in (30, 62):
            if bits <= 30:
                prm = lib.Params32(N, 1, bits=bits, device=dev)
                a, _ = synth.operands(SEED + 10, prm.q, 1, N)
                x = lib.to_device32(a, dev)
                fwd = lambda: lib.pm_ntt_fwd_u32(x, N, 1, 1, prm.q, prm.psi_br)
                inv = lambda: lib.pm_ntt_inv_u32(x, N, 1, 1, prm.q, prm.psi_inv_br)
            else:
                prm = lib.Params(N, 1, bits=bits, device=dev)
                a, _ = synth.operands(SEED + 10, prm.q, 1, N)
                x = lib.to_device(a, dev)
                fwd = lambda: lib.pm_ntt_fwd(x, N, 1, 1, prm.q, prm.psi_br)
                inv = lambda: lib.pm_ntt_inv(x, N, 1, 1, prm.q, prm.psi_inv_br)
            lat.append({"N": N, "q_bits": bits, "word_bits": 32 if bits <= 30 else 64,
                        "ntt_us": round(_graph_call_us(torch, fwd), 2),
                        "intt_us": round(_graph_call_us(torch, inv), 2),
                        "ntt_us_host_call": round(_median_call_us(torch, stream, fwd, 200), 2)})
    # same 2880-bit Q at N = 2^16, 8 pairs: 96 x 30-bit limbs on 32-bit words
    N, L32, P = 1 << 16, 96, POLYS
    prm = lib.Params32(N, L32, bits=30, device=dev)
    a, b = synth.operands(SEED + 11, prm.q, P, N)
    da, db = lib.to_device32(a, dev), lib.to_device32(b, dev)
    dc = torch.empty_like(da)
    wsb = lib.pm_polymul_u32_workspace_bytes(N, L32, P)
    ws = torch.empty(max(wsb // 4, 1), dtype=torch.int32, device=dev)

    def step():
        lib.pm_polymul_u32(da, db, dc, N, L32, P, prm.q, prm.psi_br, prm.psi_inv_br, ws)

    def with_pipeline(chunks):
        def fn():
            lib.pm_tune_set_pipeline(chunks)
            step()
        return fn

    def kernels(chunks):
        lib.pm_tune_set_pipeline(chunks)
        lib.pm_prof_read(reset=True)
        lib.pm_prof_enable(True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        lib.pm_prof_enable(False)
        return lib.pm_prof_read(reset=True)

    for _ in range(10):
        step()
    med = alternate(torch, stream, {"pipelined": with_pipeline(-1), "three_pass": with_pipeline(0)})
    ms, ms3 = med["pipelined"], med["three_pass"]
    k32, k3 = kernels(-1), kernels(0)
    lib.pm_tune_set_pipeline(-1)
    logr = N.bit_length() - 1 - 12

    def step_ops(name):
        # algorithmic ops of one step over all 96 limbs
        if name.startswith("pipe32_mul"):
            return sum(alg_ops(k, N, L32, P, OPS32[30])
                       for k in ("row32_mul_c12", "col32_fwd_r%d" % logr, "col32_inv_r%d" % logr))
        return alg_ops(name, N, L32, P, OPS32[30])

    dom = max(k32.items(), key=lambda kv: kv[1][1])[0]
    achieved = step_ops(dom) * steps / (k32[dom][1] / 1e3) / 1e12
    row3 = max(k3.items(), key=lambda kv: kv[1][1])[0]
    achieved3 = step_ops(row3) * steps / (k3[row3][1] / 1e3) / 1e12
    x = da.clone()
    ntt_us = _median_call_us(torch, stream, lambda: lib.pm_ntt_fwd_u32(x, N, L32, P, prm.q, prm.psi_br), 20)
    return {"what": "32-bit words, moduli < 2^30 (Alg. 4, beta = 32)",
            "single_transform_latency": lat,
            "polymul_96x30bit_limbs": {
                "limbs": L32, "polys_per_limb": P, "ms_per_step": round(ms, 4),
                "limb_products_per_s": round(L32 * P / ms * 1e3, 1),
                "q2880_products_per_s": round(P / ms * 1e3, 1),
                "ntt_fwd_per_s": round(L32 * P / ntt_us * 1e6, 1),
                "kernels_avg_ms": {k: round(v[1] / v[0], 4) for k, v in sorted(k32.items())},
                "roofline": {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                             "peak": round(PEAK_VALU_TOPS, 3), "unit": "TOP/s",
                             "frac": round(achieved / PEAK_VALU_TOPS, 4),
                             "ops_per_unit": {"ct": OPS32[30][0], "gs": OPS32[30][1], "mul": OPS32[30][2]}},
                "timing": "median of 4 alternating blocks of 10 steps, pipelined and three-pass",
                "three_pass": {"ms_per_step": round(ms3, 4),
                               "kernels_avg_ms": {k: round(v[1] / v[0], 4) for k, v in sorted(k3.items())},
                               "row_pass": {"kernel": row3, "achieved": round(achieved3, 3),
                                            "frac": round(achieved3 / PEAK_VALU_TOPS, 4)}}}}


def valu_issue(lib):
    """Lane-operations per second of each VALU instruction class the
    butterflies use (pm_probe_valu: 32 independent chains per thread, every CU
    busy) and the shader clock under that load."""
    rates, mhz = lib.pm_probe_valu()
    return {"clock_mhz_under_load": round(mhz, 1),
            "lane_ops_T": {k: round(v / 1e12, 2) for k, v in rates.items()},
            "peak_T_at_2400MHz_one_instruction_per_lane_per_cycle": round(PEAK_VALU_TOPS, 2),
            "what": "multiplies, v_mad_u64_u32, three-operand and carry arithmetic issue at one "
                    "instruction per lane per cycle (16 lanes per SIMD); two-operand moves and "
                    "some logic issue faster"}


def single_polymul(torch, lib, dev):
    """The latency-bound case: one product at N = 1024 under q = 2^60 - 2^14 + 1
    (the largest 60-bit prime = 1 mod 2048), device time per call from HIP-graph
    replays, with the installed small-batch plan and with the throughput plan."""
    from paper_2209_01290_amd import synth
    N = 1024
    prm = lib.Params(N, 1, device=dev)
    a, b = synth.operands(220901290 + 1, prm.q, 1, N)
    da, db = lib.to_device(a, dev), lib.to_device(b, dev)
    dc = torch.empty_like(da)
    fn = lambda: lib.pm_polymul(da, db, dc, N, 1, 1, prm.q, prm.psi_br, prm.psi_inv_br, None)
    plan = lib.pm_tune_get_small(lib.OP_POLYMUL, 10)
    out = {"what": "one N=1024 product, q = 2^60 - 2^14 + 1", "small_plan": plan,
           "device_us": round(_graph_call_us(torch, fn), 2)}
    # the throughput plan: the small-batch plan of (polymul, 2^10) removed for one measurement
    lib.pm_tune_set_small(lib.OP_POLYMUL, 10, 0, 0)
    out["device_us_throughput_plan"] = round(_graph_call_us(torch, fn), 2)
    if plan[0]:
        lib.pm_tune_set_small(lib.OP_POLYMUL, 10, *plan)
    out["host_call_us"] = round(_median_call_us(torch, torch.cuda.current_stream(dev), fn, 200), 2)
    return out


def serving(lib, rates=(2000.0, 5000.0, 10000.0, 20000.0, 50000.0), nreq=10000):
    """The continuous-batching loop on Poisson arrivals (N in 2^13..2^17,
    1..60 limbs): throughput and p50/p99 latency per offered rate."""
    from paper_2209_01290_amd import serve
    res = serve.run_rates(rates, nreq, budget_gib=32.0, streams=3, verbose=False)
    keep = ("offered_rate_req_s", "requests", "completed", "throughput_req_s", "throughput_polymul_s",
            "throughput_n16_equiv_s", "latency_ms", "mean_batch_requests", "max_queue", "max_inflight_batches",
            "arena_peak_bytes")
    return [{k: r[k] for k in keep} for r in res]


def copy_probe(torch, dev, steps):
    """Plain device-to-device copies of 1 GiB: a kernel of known HBM traffic
    (1 GiB read + 1 GiB written per launch) for scaling rocprofv3 counters."""
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    print(json.dumps({"copy_probe_bytes_read": 1 << 30, "copy_probe_bytes_written": 1 << 30,
                      "ms_per_copy": round(ms, 4), "GBps_read_plus_write": round(2 * (1 << 30) / ms / 1e6, 1)}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the batched step")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time only plain device copies of 1 GiB (calibrates HBM byte counters)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only measure the VALU issue rates and the shader clock under load")
    ap.add_argument("--words32-only", action="store_true",
                    help="run only the 32-bit word measurement (for counter runs on its kernels)")
    ap.add_argument("--part", default="all", choices=("all", "mixed", "config2", "serving"),
                    help="all: the full report; mixed / config2 / serving: only that leg "
                         "(for counter runs on its kernels)")
    ap.add_argument("--settle-s", type=float, default=2.0,
                    help="seconds of untimed steps after the warm-up, before the timed region "
                         "(lets the shader clock and power state reach steady state)")
    ap.add_argument("--pipeline-chunks", type=int, default=-1,
                    help="chunks of the software-pipelined step (-1: the library's choice; 0: three passes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the workload's limbs are independent and would be "
              "split across GPUs with no communication; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2209_01290_amd import lib, synth

    lib.load()
    tuned = lib.apply_tune_db()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        copy_probe(torch, dev, args.steps)
        return
    if args.words32_only:
        print(json.dumps({"words32": words32(torch, lib, dev, steps=args.steps)}), flush=True)
        return
    if args.valu_probe:
        print(json.dumps({"valu_issue": valu_issue(lib)}), flush=True)
        return
    if args.part == "mixed":
        print(json.dumps({"mixed_batch": mixed_batch(torch, lib, dev, launches=args.steps)}), flush=True)
        return
    if args.part == "config2":
        print(json.dumps({"config2": config2(torch, lib, dev, steps=args.steps)}), flush=True)
        return
    if args.part == "serving":
        print(json.dumps({"serving": serving(lib)}), flush=True)
        return
    lib.pm_tune_set_pipeline(args.pipeline_chunks)
    N = 1 << N_LOG2
    prm = lib.Params(N, LIMBS, device=dev)
    qs = prm.q
    a_host, b_host = synth.operands(SEED, qs, POLYS, N)
    da, db = lib.to_device(a_host, dev), lib.to_device(b_host, dev)
    dc = torch.empty_like(da)
    ws_bytes = lib.pm_polymul_workspace_bytes(N, LIMBS, POLYS)
    ws = torch.empty(max(ws_bytes // 8, 1), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        lib.pm_polymul(da, db, dc, N, LIMBS, POLYS, qs, prm.psi_br, prm.psi_inv_br, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # settle: untimed steps for a fixed time, so that the timed region starts
    # at the steady-state clock (the first few ms of load run slower)
    settle_steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < args.settle_s:
        for _ in range(25):
            step()
        torch.cuda.synchronize()
        settle_steps += 25
    settle = {"seconds": round(time.perf_counter() - t0, 3), "steps": settle_steps,
              "what": "untimed steps run for a fixed time after the warm-up steps, before the timed region"}

    # ---- timed region: K batched steps, one HIP event between steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for k in range(args.steps):
        step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    total_ms = evs[0].elapsed_time(evs[-1])
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    products = LIMBS * POLYS
    value = products * args.steps / (total_ms / 1e3)

    # ---- kernel-timing region: the same K steps with every launch bracketed
    # by HIP events on its own stream (the library's timer); the brackets add
    # a little time between kernels, so the step rate above is taken without them
    lib.pm_prof_read(reset=True)
    lib.pm_prof_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    lib.pm_prof_enable(False)
    kern = lib.pm_prof_read(reset=True)
    timed_step_ms = e0.elapsed_time(e1) / args.steps

    # ---- the same step without software pipelining (three passes: column,
    # row, column), for the row pass's own roofline
    def with_pipeline(chunks):
        def fn():
            lib.pm_tune_set_pipeline(chunks)
            step()
        return fn

    med = alternate(torch, stream, {"pipelined": with_pipeline(args.pipeline_chunks), "three_pass": with_pipeline(0)})
    lib.pm_tune_set_pipeline(0)
    lib.pm_prof_enable(True)
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    lib.pm_prof_enable(False)
    kern3 = lib.pm_prof_read(reset=True)
    lib.pm_tune_set_pipeline(args.pipeline_chunks)

    # ---- roofline of the dominant kernel (the issue ceiling is measured live
    # after the timed regions: the rates of the butterflies' instruction
    # classes and the shader clock under load)
    issue = valu_issue(lib)
    rates = {k: v * 1e12 for k, v in issue["lane_ops_T"].items()}

    def kernel_roofline(kt, name):
        launches, ms = kt[name]
        avg_s = ms / launches / 1e3
        ops = alg_ops(name, N, LIMBS, POLYS, launches_per_step=launches // args.steps)
        achieved = ops / avg_s / 1e12
        ceiling = mix_ceiling(name, N, LIMBS, POLYS, rates)
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 3),
                "unit": "TOP/s", "frac": round(achieved / PEAK_VALU_TOPS, 4),
                "traffic": measured_traffic(name), "kernel": name,
                "kernel_avg_ms": round(avg_s * 1e3, 4), "launches_per_step": launches // args.steps,
                "alg_ops_per_launch": ops, "peak_mix_measured": round(ceiling, 3),
                "frac_of_mix_measured": round(achieved / ceiling, 4)}

    dom = max(kern.items(), key=lambda kv: kv[1][1])[0]
    roofline = kernel_roofline(kern, dom)
    row3 = max(kern3.items(), key=lambda kv: kv[1][1])[0]
    three_pass = {"ms_per_step": round(med["three_pass"], 4),
                  "value": round(products / med["three_pass"] * 1e3, 1), "unit": "polymul/s",
                  "pipelined_ms_per_step_alternating": round(med["pipelined"], 4),
                  "pipelined_over_three_pass": round(med["three_pass"] / med["pipelined"], 4),
                  "timing": "median of 4 alternating blocks of 10 steps, pipelined and three-pass",
                  "kernels_avg_ms": {k: round(v[1] / v[0], 4) for k, v in sorted(kern3.items())},
                  "row_pass_roofline": kernel_roofline(kern3, row3),
                  "what": "the same step with pm_tune_set_pipeline(0): column pass, row pass, "
                          "column pass as three launches"}
    # HBM view of the whole step: operands and result once, tables once per limb
    b_alg = products * 24 * N + LIMBS * 16 * N
    hbm = {"alg_bytes_per_step": b_alg,
           "achieved_GBps": round(b_alg * args.steps / (total_ms / 1e3) / 1e9, 1),
           "peak_GBps": PEAK_HBM_GBPS}
    hbm["frac"] = round(hbm["achieved_GBps"] / PEAK_HBM_GBPS, 4)

    out = {
        "metric": "negacyclic polymul/s & % HBM roofline, N=2^16 q<2^60; batched vs plain; p99",
        "value": round(value, 1), "unit": "polymul/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "N=2^16 negacyclic polymul, 48 limbs x 8 pairs (384 products), "
                               "48 largest 60-bit primes q = 1 mod 2^17, uniform operands",
                   "N": N, "limbs": LIMBS, "polys_per_limb": POLYS, "path": "pm_polymul (batched)",
                   "pass_plan_logc": lib.pm_tune_get(lib.OP_POLYMUL, N_LOG2),
                   "tuned_entries": tuned},
        "latency_ms": {"p50": round(pct(step_ms, 50), 4), "p99": round(pct(step_ms, 99), 4),
                       "unit": "per batched step of 384 products"},
        "step_ms": [round(x, 4) for x in step_ms],
        "settle": settle,
        "pipeline_chunks": lib.pm_tune_get_pipeline(),
        "roofline": roofline,
        "three_pass": three_pass,
        "valu_issue": issue,
        "hbm_roofline": hbm,
        "kernels_avg_ms": {k: round(v[1] / v[0], 4) for k, v in sorted(kern.items())},
        "kernel_timing": {"steps": args.steps, "ms_per_step_with_kernel_timer": round(timed_step_ms, 4)},
    }

    if not args.no_extra:
        # plain: one launch sequence per product
        plain_ms = []
        for _ in range(1 + args.plain_steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(products + 1)]
            ev[0].record(stream)
            i = 0
            for l in range(LIMBS):
                for p in range(POLYS):
                    lib.pm_polymul(da[l, p], db[l, p], dc[l, p], N, 1, 1, [qs[l]], prm.psi_br[l],
                                   prm.psi_inv_br[l], ws)
                    i += 1
                    ev[i].record(stream)
            torch.cuda.synchronize()
            plain_ms.append([ev[k].elapsed_time(ev[k + 1]) for k in range(products)])
        per = [x for run in plain_ms[1:] for x in run]
        out["plain"] = {"value": round(1e3 / (sum(per) / len(per)), 1), "unit": "polymul/s",
                        "p50_ms": round(pct(per, 50), 4), "p99_ms": round(pct(per, 99), 4),
                        "what": "384 separate pm_polymul calls per step (one launch sequence each)"}
        out["batched_over_plain"] = round(value / out["plain"]["value"], 3)
        # the fused product of Sec. III-B (Alg. 8) on the same batch, in
        # alternating blocks of 10 steps with the Eq. 2 step (same clocks)
        def fstep():
            lib.pm_polymul_fused(da, db, dc, N, LIMBS, POLYS, qs, prm.psi_br, prm.psi_inv_br, ws)
        blocks = {"eq2": [], "fused": []}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(4):
            for name, fn in (("eq2", step), ("fused", fstep)):
                for _ in range(2):
                    fn()
                e0.record(stream)
                for _ in range(10):
                    fn()
                e1.record(stream)
                torch.cuda.synchronize()
                blocks[name].append(e0.elapsed_time(e1) / 10)
        lib.pm_prof_read(reset=True)
        lib.pm_prof_enable(True)
        for _ in range(10):
            fstep()
        torch.cuda.synchronize()
        lib.pm_prof_enable(False)
        fk = lib.pm_prof_read(reset=True)
        f_ms, q_ms = pct(blocks["fused"], 50), pct(blocks["eq2"], 50)
        out["fused"] = {"value": round(products / f_ms * 1e3, 1), "unit": "polymul/s",
                        "ms_per_step": round(f_ms, 4), "eq2_ms_per_step_alternating": round(q_ms, 4),
                        "fused_over_eq2": round(q_ms / f_ms, 4),
                        "what": "pm_polymul_fused (Alg. 8: truncated NTTs + Karatsuba-fused Hadamard), "
                                "median of 4 blocks of 10 steps alternating with the Eq. 2 step",
                        "kernels_avg_ms": {k: round(v[1] / v[0], 4) for k, v in sorted(fk.items())}}
        # stagewise: one launch per NTT stage, whole batch per launch
        sws = torch.empty(lib.pm_polymul_stagewise_workspace_bytes(N, LIMBS, POLYS) // 8,
                          dtype=torch.int64, device=dev)
        for _ in range(2):
            lib.pm_polymul_stagewise(da, db, dc, N, LIMBS, POLYS, qs, prm.psi_br, prm.psi_inv_br, sws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 3
        for _ in range(reps):
            lib.pm_polymul_stagewise(da, db, dc, N, LIMBS, POLYS, qs, prm.psi_br, prm.psi_inv_br, sws)
        e1.record(stream)
        torch.cuda.synchronize()
        out["stagewise"] = {"value": round(products * reps / (e0.elapsed_time(e1) / 1e3), 1),
                            "unit": "polymul/s", "what": "pm_polymul_stagewise, one launch per stage"}
        del sws
        # standalone forward NTT of the 384 a operands
        x = da.clone()
        for _ in range(3):
            lib.pm_ntt_fwd(x, N, LIMBS, POLYS, qs, prm.psi_br)
        e0.record(stream)
        reps = 20
        for _ in range(reps):
            lib.pm_ntt_fwd(x, N, LIMBS, POLYS, qs, prm.psi_br)
        e1.record(stream)
        torch.cuda.synchronize()
        out["ntt_fwd"] = {"value": round(products * reps / (e0.elapsed_time(e1) / 1e3), 1),
                          "unit": "NTT/s", "what": "pm_ntt_fwd over the 384 a operands"}
        # restore the batched result for the CPU check below
        step()
        torch.cuda.synchronize()
        out["mixed_batch"] = mixed_batch(torch, lib, dev)
        out["mixed_batch"]["over_uniform_step_n16_rate"] = round(out["mixed_batch"]["n16_equivalent_per_s"] / value, 4)
        out["single_polymul_n1024"] = single_polymul(torch, lib, dev)
        w32 = words32(torch, lib, dev)
        w32["polymul_96x30bit_limbs"]["vs_48x60bit_limbs_u64"] = round(
            w32["polymul_96x30bit_limbs"]["q2880_products_per_s"] / (value / LIMBS), 3)
        out["words32"] = w32
        out["config2"] = config2(torch, lib, dev)
        out["serving"] = serving(lib)

    if not args.no_cpu:
        gpu_c = lib.to_host(dc).reshape(a_host.shape)
        out["cpu_baseline"] = cpu_baseline(N, qs, a_host, b_host, gpu_c)
        out["gpu_over_cpu"] = round(value / out["cpu_baseline"]["value"], 1)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
