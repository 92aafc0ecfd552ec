"""Barrett variant study on the device (Sec. II-B, Fig. 4 and the correction
statistics): for 32-bit words (28/29/30-bit moduli) and 64-bit words (up to
62-bit moduli), the classical reduction (Alg. 2), Dhem-Quisquater alpha = N+3
(Alg. 3), the proposed variant (Alg. 4) and the built-in '%':

  * throughput: reductions per second of 8 independent chains x <- reduce(x*y)
    per thread over `iters` steps (the paper times one reduction averaged over
    10,000 iterations);
  * correction statistics: share of reductions needing 0 / 1 / 2 correctional
    subtractions on uniform products a*b, a, b uniform in [0, q).

Moduli: the largest prime q < 2^bits with q = 1 mod 2048.

Usage on a GPU:  python -m paper_2209_01290_amd.barrett_study [--iters 10000]
"""
from __future__ import annotations

import argparse
import json

NAMES = {0: "%", 2: "Alg2 classical", 3: "Alg3 DQ(N+3)", 4: "Alg4 proposed"}
CASES = [(32, 28), (32, 29), (32, 30), (64, 28), (64, 30), (64, 60), (64, 62)]


def valid(variant: int, word_bits: int, qbits: int) -> bool:
    if variant == 3:
        return qbits <= word_bits - 4
    if variant in (2, 4):
        return qbits <= word_bits - 2
    return qbits <= (32 if word_bits == 32 else 62)


def study(iters: int = 10000, threads: int = 65536, pairs: int = 1 << 20, verbose=True):
    import torch
    from . import lib, synth
    lib.load()
    dev = torch.device("cuda")
    out = torch.empty(threads, dtype=torch.int64, device=dev)
    rows = []
    for word_bits, qbits in CASES:
        q = lib.pm_ntt_primes(1024, 1, qbits)[0]
        a = lib.to_device(synth.uniform_mod(synth.key(31, qbits, 0), pairs, q), dev)
        b = lib.to_device(synth.uniform_mod(synth.key(31, qbits, 1), pairs, q), dev)
        c = torch.empty_like(a)
        hist = torch.zeros(3 * ((pairs + 255) // 256), dtype=torch.int32, device=dev)
        y = (q * 2) // 3
        for variant in (0, 2, 3, 4):
            if not valid(variant, word_bits, qbits):
                continue
            lib.pm_reduce_chain(variant, word_bits, out, y, 10, q)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lib.pm_reduce_chain(variant, word_bits, out, y, iters, q)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            red = threads * 8.0 * iters
            hist.zero_()
            lib.pm_reduce_apply(variant, word_bits, a, b, c, hist, q)
            torch.cuda.synchronize()
            h = hist.view(-1, 3).sum(dim=0).cpu().tolist()
            row = {"word_bits": word_bits, "q_bits": qbits, "q": q, "variant": NAMES[variant],
                   "reductions_per_s": red / ms * 1e3, "ns_per_reduction_per_lane":
                       ms * 1e6 / (iters * 8.0) if threads else None,
                   "corrections_pct": [round(100.0 * x / pairs, 3) for x in h]}
            rows.append(row)
            if verbose:
                print(json.dumps(row), flush=True)
    return rows


def markdown(rows) -> str:
    md = ["| word | q bits | variant | G reductions/s | ns per reduction (per lane chain) | "
          "0 / 1 / 2 corrections (%) |", "|---|---|---|---|---|---|"]
    for r in rows:
        md.append("| %d | %d | %s | %.1f | %.3f | %s |" % (
            r["word_bits"], r["q_bits"], r["variant"], r["reductions_per_s"] / 1e9,
            r["ns_per_reduction_per_lane"], " / ".join("%.2f" % x for x in r["corrections_pct"])))
    return "\n".join(md) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=10000)
    ap.add_argument("--out", default=None, help="write the rows as JSON here")
    a = ap.parse_args()
    rows = study(a.iters)
    print(markdown(rows), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
