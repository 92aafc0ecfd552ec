"""Autotuner for the pass plan of each transform size.

For every N and operation (pm_polymul, pm_ntt_fwd, pm_ntt_inv) it times
every split the kernels implement -- rows of 2^logc words in LDS after a
column pass of radix R = N / 2^logc in registers, or a single row pass when
logc = log2 N -- on a batch large enough to fill the GPU, installs the fastest
with pm_tune_set and writes the choices to a JSON database:

    {"arch": "gfx950", "device": "...", "choices": {"polymul": {"16": 12, ...}, ...},
     "timings_ms": {"polymul": {"16": {"12": 0.81, "13": 0.85}, ...}, ...}}

Usage on a GPU:  python -m paper_2209_01290_amd.tune [--out FILE] [--log2n 12-17]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_DB)
    ap.add_argument("--log2n", default="1-17", help="range lo-hi of log2 N")
    a = ap.parse_args()
    lo, hi = (int(v) for v in a.log2n.split("-"))
    db = tune(range(lo, hi + 1))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(db, f, indent=1)
    print("[tune] wrote " + a.out, flush=True)


if __name__ == "__main__":
    main()
