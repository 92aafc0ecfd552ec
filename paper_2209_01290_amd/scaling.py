"""Weak-scaling study of the transforms on one GPU (Sec. V-C and the
single-block scaling experiment of Sec. VI), in both batch layouts:

  * batch scaling (the throughput-optimised multi-block design): forward
    NTTs of N = 2^16 under one 60-bit modulus, the batch doubled from 1 to
    2^15 polynomials (the paper's largest shape: 2^15 transforms of 2^16
    points), each batch one call; time per call and per transform, in the
    [poly][N] layout (pm_ntt_fwd) and the coefficient-major [N][poly] layout
    (pm_ntt_fwd_il);
  * single-transform scaling: one forward NTT of N = 2^10 .. 2^17, where the
    number of workgroups grows with N (the paper doubles N and the block
    count together): device time per call (20 calls captured in one HIP
    graph, replayed), and the time per call when launched from Python.

Operands: uniform in [0, q) from the seeded device generator. Every timing is
the median of HIP-event intervals between consecutive calls on one stream.

Usage on a GPU:  python -m paper_2209_01290_amd.scaling [--max-log2p 15] [--out F]
                 [--single [--log2n 10-17]]   (single transforms only)
"""
from __future__ import annotations

import argparse
import json

SEED = 220901290 + 9


def _median_us(torch, fn, reps):
    stream = torch.cuda.current_stream()
    for _ in range(3):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(reps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    xs = sorted(ev[k].elapsed_time(ev[k + 1]) * 1e3 for k in range(reps))
    return xs[len(xs) // 2]


def _graph_us(torch, fn, calls=20, reps=10):
    """Device time of one call without host overhead: `calls` consecutive calls
    captured in one HIP graph, replayed `reps` times; median per call."""
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


def batch_scaling(torch, lib, log2n=16, max_log2p=15, verbose=True):
    from . import synth
    dev = torch.device("cuda")
    N = 1 << log2n
    prm = lib.Params(N, 1, device=dev)
    rows = []
    for lp in range(0, max_log2p + 1):
        P = 1 << lp
        x = torch.empty(P * N, dtype=torch.int64, device=dev)
        chunk = min(P * N, 1 << 24)          # drawn 2^24 words at a time (stream = chunk index)
        for c in range(P * N // chunk):
            synth.uniform_mod_device([synth.key(SEED, lp, c)], chunk, prm.q, x[c * chunk:(c + 1) * chunk].view(1, chunk))
        reps = max(5, min(200, (1 << 22) // (P * N // 64 + 1)))
        row = {"N": N, "polys": P, "bytes": P * N * 8}
        # HBM bytes each layout moves per call: every pass reads and writes the batch once
        std_passes = 2 if lib.pm_tune_get(lib.OP_NTT_FWD, log2n) < log2n else 1
        il_passes = -(-log2n // 6)            # blocks of at most 6 stages
        moved = {"standard": std_passes * 16 * N * P, "interleaved": il_passes * 16 * N * P}
        for name, fn in (("standard", lambda: lib.pm_ntt_fwd(x, N, 1, P, prm.q, prm.psi_br)),
                         ("interleaved", lambda: lib.pm_ntt_fwd_il(x, N, 1, P, prm.q, prm.psi_br))):
            us = _median_us(torch, fn, reps)
            row[name + "_us_per_call"] = round(us, 2)
            row[name + "_us_per_ntt"] = round(us / P, 4)
            row[name + "_GBps"] = round(moved[name] / us / 1e3, 1)
        rows.append(row)
        if verbose:
            print(json.dumps(row), flush=True)
        del x
        torch.cuda.empty_cache()
    return rows


def single_scaling(torch, lib, verbose=True, log2ns=range(10, 18)):
    from . import synth
    dev = torch.device("cuda")
    rows = []
    for log2n in log2ns:
        N = 1 << log2n
        prm = lib.Params(N, 1, device=dev)
        a, _ = synth.operands(SEED, prm.q, 1, N)
        x = lib.to_device(a, dev)
        fwd = lambda: lib.pm_ntt_fwd(x, N, 1, 1, prm.q, prm.psi_br)
        inv = lambda: lib.pm_ntt_inv(x, N, 1, 1, prm.q, prm.psi_inv_br)
        row = {"N": N, "ntt_us": round(_graph_us(torch, fwd), 2), "intt_us": round(_graph_us(torch, inv), 2),
               "ntt_us_host_call": round(_median_us(torch, fwd, 200), 2)}
        rows.append(row)
        if verbose:
            print(json.dumps(row), flush=True)
    return rows


def markdown(batch, single) -> str:
    md = ["| N | polys | [poly][N]: us/call | us/NTT | GB/s | [N][poly]: us/call | us/NTT | GB/s |",
          "|---|---|---|---|---|---|---|---|"]
    for r in batch:
        md.append("| 2^%d | %d | %.1f | %.4f | %.0f | %.1f | %.4f | %.0f |" % (
            r["N"].bit_length() - 1, r["polys"], r["standard_us_per_call"], r["standard_us_per_ntt"],
            r["standard_GBps"], r["interleaved_us_per_call"], r["interleaved_us_per_ntt"], r["interleaved_GBps"]))
    md += ["", "| N | one NTT (us, device) | one iNTT (us, device) | one NTT launched from Python (us) |",
           "|---|---|---|---|"]
    for r in single:
        md.append("| 2^%d | %.2f | %.2f | %.2f |" % (r["N"].bit_length() - 1, r["ntt_us"], r["intt_us"],
                                                   r["ntt_us_host_call"]))
    return "\n".join(md) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-log2p", type=int, default=15)
    ap.add_argument("--out", default=None)
    ap.add_argument("--single", action="store_true", help="only the single-transform scaling")
    ap.add_argument("--log2n", default="10-17", help="range lo-hi of log2 N for the single transforms")
    a = ap.parse_args()
    import torch
    from . import lib
    lib.load()
    lib.apply_tune_db()
    lo, hi = (int(v) for v in a.log2n.split("-"))
    single = single_scaling(torch, lib, log2ns=range(lo, hi + 1))
    batch = [] if a.single else batch_scaling(torch, lib, max_log2p=a.max_log2p)
    print(markdown(batch, single), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"batch": batch, "single": single}, f, indent=1)


if __name__ == "__main__":
    main()
