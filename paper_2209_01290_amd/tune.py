"""Autotuner for the pass plan of each transform size.

For every N and operation (pm_polymul, pm_ntt_fwd, pm_ntt_inv) it times
every split the kernels implement -- rows of 2^logc words in LDS after a
column pass of radix R = N / 2^logc in registers, or a single row pass when
logc = log2 N -- on a batch large enough to fill the GPU, installs the fastest
with pm_tune_set and writes the choices to a JSON database:

    {"arch": "gfx950", "device": "...", "choices": {"polymul": {"16": 12, ...}, ...},
     "timings_ms": {"polymul": {"16": {"12": 0.81, "13": 0.85}, ...}, ...}}

Small-batch plans (--small): for a single transform or product per call
(one limb, one polynomial) it times every split with 16 and with 4 words per
thread (device time per call, 20 calls captured in one HIP graph and
replayed), keeps the fastest per (operation, N), and finds for each
(operation, N >= 2^8) the largest batch (in words) at which the small-batch
plan still beats the throughput plan, doubling the batch from one
polynomial; the smallest of these limits is the global threshold W for the
other sizes:

    "small": {"max_words": W, "choices": {"polymul": {"16": [logc, words_per_thread]}, ...},
              "limits": {"polymul": {"16": words, ...}, ...},
              "latency_us": {...}, "crossover_us": {...}}

Pipelining thresholds (--pipeline): for N = 2^15..2^17 (rows of 2^12 words
after a column pass of radix 2^3..2^5) the product over 16..480 products is
timed with the software pipeline (two chunks) and with three passes in
alternating blocks; per radix, the row count from which pipelining every
larger batch minimises the summed relative time over the measured batches:

    "pipeline": {"min_rows": {"3": rows, "4": rows, "5": rows}, "timings_ms": {...}}

Usage on a GPU:  python -m paper_2209_01290_amd.tune [--out FILE] [--log2n 12-17] [--small | --pipeline]
Applying a database: lib.apply_tune_db(FILE) (bench.py and serve.py do).
"""
from __future__ import annotations

import argparse
import json
import os

OPS = {"polymul": 2, "ntt_fwd": 0, "ntt_inv": 1}
DEFAULT_DB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_db", "gfx950.json")


def candidates(log2n: int):
    """logc values with an implemented split: single pass up to 2^14 words,
    else rows of >= 2^8 words and a column radix of at most 2^5."""
    out = []
    for logc in range(1, min(log2n, 14) + 1):
        R = log2n - logc
        if R == 0 or (R <= 5 and logc >= 8):
            out.append(logc)
    return out


def _time(torch, fn, reps=8, warm=3):
    for _ in range(warm):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(log2ns, words=1 << 25, device="cuda", verbose=True):
    import torch
    from . import lib, synth
    lib.load()
    dev = torch.device(device)
    # time the throughput plans only: no small-batch plan may take a call
    for op in OPS.values():
        for n in range(1, 18):
            lib.pm_tune_set_small(op, n, 0, 0)
    choices = {k: {} for k in OPS}
    timings = {k: {} for k in OPS}
    for log2n in log2ns:
        N = 1 << log2n
        total = max(1, words // N)                 # polynomials per operand
        limbs = min(64, total)
        polys = min(65535, max(1, total // limbs))
        prm = lib.Params(N, limbs, device=dev)
        a, b = synth.operands(synth.SEED_BASE + 17, prm.q, 1, N)
        da = lib.to_device(a, dev).repeat(1, polys, 1).contiguous()
        db = lib.to_device(b, dev).repeat(1, polys, 1).contiguous()
        dc = torch.empty_like(da)
        x = da.clone()
        for name, op in OPS.items():
            best, best_ms = None, None
            timings[name][str(log2n)] = {}
            for logc in candidates(log2n):
                lib.pm_tune_set(op, log2n, logc)
                nbytes = lib.pm_polymul_workspace_bytes(N, limbs, polys)
                ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device=dev)
                if name == "polymul":
                    fn = lambda: lib.pm_polymul(da, db, dc, N, limbs, polys, prm.q, prm.psi_br, prm.psi_inv_br, ws)
                elif name == "ntt_fwd":
                    fn = lambda: lib.pm_ntt_fwd(x, N, limbs, polys, prm.q, prm.psi_br)
                else:
                    fn = lambda: lib.pm_ntt_inv(x, N, limbs, polys, prm.q, prm.psi_inv_br)
                ms = _time(torch, fn)
                timings[name][str(log2n)][str(logc)] = round(ms, 4)
                if best_ms is None or ms < best_ms:
                    best, best_ms = logc, ms
                del ws
            lib.pm_tune_set(op, log2n, best)
            choices[name][str(log2n)] = best
            if verbose:
                print("[tune] %-8s N=2^%-2d -> logc=%d  %s" % (name, log2n, best, timings[name][str(log2n)]),
                      flush=True)
        del da, db, dc, x
    props = torch.cuda.get_device_properties(dev)
    return {"arch": getattr(props, "gcnArchName", "gfx950").split(":")[0], "device": props.name,
            "batch_words": words, "choices": choices, "timings_ms": timings}


def small_candidates(log2n: int):
    """(logc, words_per_thread) pairs of the small-batch plans: the throughput
    splits with 16 words per thread, and with 4 words per thread rows of
    2^5..2^12 words over a column pass of 2^2..2^7 rows (2 rows only with
    >= 2^8 columns)."""
    out = [(c, 16) for c in candidates(log2n)]
    for c in range(5, min(log2n, 12) + 1):
        r = log2n - c
        if r <= 7 and not (r == 1 and c < 8):
            out.append((c, 4))
    return out


def _graph_us(torch, fn, calls=20, reps=5):
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        g.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) * 1e3 / calls for k in range(reps))
    del g
    return per[len(per) // 2]


def _calls(lib, name, prm, N, polys, da, db, dc, x, ws):
    if name == "polymul":
        return lambda: lib.pm_polymul(da, db, dc, N, 1, polys, prm.q, prm.psi_br, prm.psi_inv_br, ws)
    if name == "ntt_fwd":
        return lambda: lib.pm_ntt_fwd(x, N, 1, polys, prm.q, prm.psi_br)
    return lambda: lib.pm_ntt_inv(x, N, 1, polys, prm.q, prm.psi_inv_br)


LIMIT_MIN_LOG2N = 8            # per-N limits for N >= 2^8; the global threshold below
LIMIT_MAX_WORDS = 1 << 24      # largest batch the limit search tries (128 MiB per operand)
UNLIMITED = (1 << 64) - 1      # limit recorded when the small plan still wins at LIMIT_MAX_WORDS


def tune_small(log2ns, device="cuda", verbose=True):
    import torch
    from . import lib, synth
    lib.load()
    dev = torch.device(device)
    lib.pm_tune_set_small_batch(1 << 40)          # every call below is "small" while tuning
    for op in OPS.values():
        for n in range(1, 18):
            lib.pm_tune_set_small_limit(op, n, 0)
    choices = {k: {} for k in OPS}
    lat = {k: {} for k in OPS}
    for log2n in log2ns:
        if log2n < 5:
            continue
        N = 1 << log2n
        prm = lib.Params(N, 1, device=dev)
        a, b = synth.operands(synth.SEED_BASE + 18, prm.q, 1, N)
        da, db = lib.to_device(a, dev), lib.to_device(b, dev)
        dc = torch.empty_like(da)
        x = da.clone()
        for name, op in OPS.items():
            lat[name][str(log2n)] = {}
            best, best_us = None, None
            for logc, wpt in small_candidates(log2n):
                lib.pm_tune_set_small(op, log2n, logc, wpt)
                nbytes = lib.pm_polymul_workspace_bytes(N, 1, 1)
                ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device=dev)
                us = _graph_us(torch, _calls(lib, name, prm, N, 1, da, db, dc, x, ws))
                lat[name][str(log2n)]["%d/%d" % (logc, wpt)] = round(us, 2)
                if best_us is None or us < best_us:
                    best, best_us = (logc, wpt), us
            lib.pm_tune_set_small(op, log2n, *best)
            choices[name][str(log2n)] = list(best)
            if verbose:
                print("[tune-small] %-8s N=2^%-2d -> %s  %.2f us  %s" % (name, log2n, best, best_us,
                                                                    lat[name][str(log2n)]), flush=True)
    # Per-(op, N) limit: the largest batch (polynomials doubled from 1, up to
    # LIMIT_MAX_WORDS words) at which the small plan still beats the
    # throughput plan; the search stops after two sizes in a row lost. A plan
    # that still wins at the largest size (the GPU long full, the time per
    # polynomial steady) has no limit.
    cross = {}
    limits = {k: {} for k in OPS}
    for log2n in log2ns:
        if log2n < LIMIT_MIN_LOG2N or str(log2n) not in choices["polymul"]:
            continue
        N = 1 << log2n
        prm = lib.Params(N, 1, device=dev)
        pmax = min(LIMIT_MAX_WORDS // N, 1 << 15)       # at most 65535 polynomials per call
        a, b = synth.operands(synth.SEED_BASE + 19, prm.q, pmax, N)
        da_all, db_all = lib.to_device(a, dev), lib.to_device(b, dev)
        for name, op in OPS.items():
            keep = lib.pm_tune_get_small(op, log2n)
            won, lost, polys = 0, 0, 1
            while polys <= pmax and lost < 2:
                da, db = da_all[:, :polys].contiguous(), db_all[:, :polys].contiguous()
                dc = torch.empty_like(da)
                x = da.clone()
                t = {}
                for label, plan in (("small", keep), ("throughput", (0, 0))):
                    lib.pm_tune_set_small(op, log2n, *plan)
                    nbytes = lib.pm_polymul_workspace_bytes(N, 1, polys)
                    ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device=dev)
                    t[label] = round(_graph_us(torch, _calls(lib, name, prm, N, polys, da, db, dc, x, ws)), 2)
                lib.pm_tune_set_small(op, log2n, *keep)
                cross["%s/%d/%d" % (name, log2n, polys)] = t
                if t["small"] < t["throughput"]:
                    won, lost = N * polys, 0
                else:
                    lost += 1
                polys *= 2
            if won == N * pmax:
                won = UNLIMITED
            limits[name][str(log2n)] = won
            lib.pm_tune_set_small_limit(op, log2n, won)
            if verbose:
                print("[tune-small] limit %-8s N=2^%-2d: small plan up to %d words" % (name, log2n, won), flush=True)
    # the global threshold (for N without a limit): the smallest limit
    max_words = min((w for t in limits.values() for w in t.values()), default=0)
    max_words = min(max_words, LIMIT_MAX_WORDS)
    lib.pm_tune_set_small_batch(max_words)
    return {"max_words": max_words, "choices": choices, "limits": limits, "latency_us": lat,
            "crossover_us": cross}


# batch shapes (limbs, pairs per limb): 16..480 products
PIPE_SHAPES = ((16, 1), (32, 1), (48, 1), (48, 2), (48, 3), (48, 4), (48, 5), (48, 6), (48, 8), (48, 10))
NEVER = (1 << 64) - 1


def tune_pipeline(log2ns=(15, 16, 17), shapes=PIPE_SHAPES, device="cuda", verbose=True, reps=4, calls=10):
    """The threshold of the default software pipelining, per column radix
    2^logr (N = 2^(12 + logr), rows of 2^12 words): for each batch shape the
    product is timed with two chunks and with three passes in alternating
    blocks, after the tuned plans are installed; the threshold is the row
    count (products x 2^logr) from which pipelining every larger measured
    batch gives the least summed time over all measured batches, each
    relative to its three-pass time (never, if no threshold beats three
    passes everywhere). Installs the thresholds with
    pm_tune_set_pipeline_rows."""
    import time
    import torch
    from . import lib, synth
    lib.load()
    lib.apply_tune_db()
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev)
    min_rows, timings = {}, {}
    for log2n in log2ns:
        N, logr = 1 << log2n, log2n - 12
        res = {}
        for limbs, polys in shapes:
            P = limbs * polys
            prm = lib.Params(N, limbs, device=dev)
            a, b = synth.operands(synth.SEED_BASE + 19, prm.q, 1, N)
            da = lib.to_device(a, dev).repeat(1, polys, 1).contiguous()
            db = lib.to_device(b, dev).repeat(1, polys, 1).contiguous()
            dc = torch.empty_like(da)
            ws = torch.empty(max(lib.pm_polymul_workspace_bytes(N, limbs, polys) // 8, 1), dtype=torch.int64,
                             device=dev)

            def step():
                lib.pm_polymul(da, db, dc, N, limbs, polys, prm.q, prm.psi_br, prm.psi_inv_br, ws)

            t0 = time.perf_counter()
            while time.perf_counter() - t0 < 0.3:       # settle the clock
                for _ in range(calls):
                    step()
                torch.cuda.synchronize()
            per = {0: [], 2: []}
            for _ in range(reps):
                for g in (0, 2):
                    lib.pm_tune_set_pipeline(g)
                    step()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(calls):
                        step()
                    e1.record(stream)
                    torch.cuda.synchronize()
                    per[g].append(e0.elapsed_time(e1) / calls)
            lib.pm_tune_set_pipeline(-1)
            three, pipe = sorted(per[0])[reps // 2], sorted(per[2])[reps // 2]
            res[P] = (three, pipe)
            if verbose:
                print("[tune-pipe] N=2^%d %4d products (%6d rows): three-pass %.4f ms, two chunks %.4f ms (%.3fx)"
                      % (log2n, P, P << logr, three, pipe, three / pipe), flush=True)
            del da, db, dc, ws
        # the threshold that minimises the summed time of the measured batch
        # sizes, each relative to its three-pass time (so that every size
        # counts alike): batches from the threshold up run pipelined
        rows, best = NEVER, float(len(res))
        for cut in sorted(res):
            cost = sum(1.0 if P < cut else pipe / three for P, (three, pipe) in res.items())
            if cost < best - 1e-9:
                rows, best = cut << logr, cost
        lib.pm_tune_set_pipeline_rows(logr, rows)
        min_rows[str(logr)] = rows
        timings[str(log2n)] = {str(P): [round(t, 4), round(p, 4)] for P, (t, p) in res.items()}
        if verbose:
            print("[tune-pipe] N=2^%d: pipelined from %s rows" % (log2n, "never" if rows == NEVER else rows),
                  flush=True)
    return {"min_rows": min_rows, "timings_ms": timings,
            "what": "per column radix 2^logr: rows of 2^12 words from which two chunks beat three passes; "
                    "timings [three-pass, two chunks] ms per call by products"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_DB)
    ap.add_argument("--log2n", default="1-17", help="range lo-hi of log2 N")
    ap.add_argument("--small", action="store_true",
                    help="tune only the small-batch plans and merge them into --out")
    ap.add_argument("--pipeline", action="store_true",
                    help="tune only the thresholds of the software-pipelined product and merge them into --out")
    a = ap.parse_args()
    lo, hi = (int(v) for v in a.log2n.split("-"))
    if a.pipeline:
        db = json.load(open(a.out)) if os.path.exists(a.out) else {}
        db["pipeline"] = tune_pipeline()
        with open(a.out, "w") as f:
            json.dump(db, f, indent=1)
        print("[tune] wrote " + a.out, flush=True)
        return
    if a.small:
        db = json.load(open(a.out)) if os.path.exists(a.out) else {}
        db["small"] = tune_small(range(lo, hi + 1))
        with open(a.out, "w") as f:
            json.dump(db, f, indent=1)
        print("[tune] wrote " + a.out, flush=True)
        return
    db = tune(range(lo, hi + 1))
    if os.path.exists(a.out):
        old = json.load(open(a.out))
        for part in ("small", "pipeline"):      # tuned separately
            if part in old:
                db[part] = old[part]
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(db, f, indent=1)
    print("[tune] wrote " + a.out, flush=True)


if __name__ == "__main__":
    main()
