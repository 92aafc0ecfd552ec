"""Seeded synthetic workloads, laid out on the device.

mixed_requests   request shapes of the batched mixed workload: N uniform on
                 2^12..2^17, L (limbs) uniform on 1..48
serving_requests Poisson arrivals for the serving loop: N in 2^13..2^17 with
                 weights .1/.2/.3/.25/.15, L uniform on 1..60
MixedBatch       one request list resident on the device: operands drawn with
                 the device generator, moduli and twiddle tables per (N, limb),
                 and one pm_job per (request, limb).

Limb l of a size-N request uses the l-th largest prime q < 2^60 with
q = 1 mod 2N. Operand streams are keyed (seed, request, limb, 0, a/b).
Every draw here comes from the SplitMix64 generator of ``synth`` (integer
draws by reduction of a 64-bit word, uniform up to a bias below 2^-58).
"""
from __future__ import annotations

import math

import numpy as np

from . import synth

META = 0x5EED


def _meta_words(seed: int, n: int) -> np.ndarray:
    return synth.words(synth.key(seed, META), n)


def mixed_requests(seed: int, nreq: int = 512, lo: int = 12, hi: int = 17, max_limbs: int = 48):
    w = _meta_words(seed, 2 * nreq)
    span = hi - lo + 1
    return [(lo + int(w[2 * r] % np.uint64(span)), 1 + int(w[2 * r + 1] % np.uint64(max_limbs)))
            for r in range(nreq)]


SERVE_LOG2N = (13, 14, 15, 16, 17)
SERVE_WEIGHTS = (0.10, 0.20, 0.30, 0.25, 0.15)


def serving_requests(seed: int, nreq: int, rate: float, max_limbs: int = 60):
    """[(arrival_s, log2n, L)]: exponential inter-arrival times at `rate`/s."""
    w = _meta_words(seed, 3 * nreq)
    u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    cum = np.cumsum(SERVE_WEIGHTS)
    out, t = [], 0.0
    for r in range(nreq):
        t += -math.log(1.0 - u[3 * r]) / rate
        k = int(np.searchsorted(cum, u[3 * r + 1], side="right"))
        L = 1 + int(w[3 * r + 2] % np.uint64(max_limbs))
        out.append((t, SERVE_LOG2N[min(k, len(SERVE_LOG2N) - 1)], L))
    return out


class Tables:
    """Device-resident moduli and twiddle tables per N (limbs on demand)."""

    def __init__(self, device):
        self.device = device
        self.by_n = {}

    def get(self, log2n: int, limbs: int):
        from . import lib
        have = self.by_n.get(log2n)
        if have is None or len(have.q) < limbs:
            have = lib.Params(1 << log2n, max(limbs, len(have.q) if have else 0), device=self.device)
            self.by_n[log2n] = have
        return have


class MixedBatch:
    """Operands a, b and outputs c of a request list, one [S, N] block per N."""

    def __init__(self, requests, seed: int, device, tables: Tables | None = None, chunk: int = 64):
        import torch
        from . import lib
        self.requests = list(requests)
        self.seed = seed
        self.device = device
        self.tables = tables or Tables(device)
        self.slot = {}                 # (request, limb) -> (log2n, row)
        rows = {}
        for r, (log2n, L) in enumerate(self.requests):
            for l in range(L):
                self.slot[(r, l)] = (log2n, rows.get(log2n, 0))
                rows[log2n] = rows.get(log2n, 0) + 1
        self.a, self.b, self.c = {}, {}, {}
        for log2n, S in rows.items():
            N = 1 << log2n
            maxl = max(L for (n2, L) in self.requests if n2 == log2n)
            prm = self.tables.get(log2n, maxl)
            a = torch.empty((S, N), dtype=torch.int64, device=device)
            b = torch.empty((S, N), dtype=torch.int64, device=device)
            keys_a, keys_b, qs = [], [], []
            for (r, l), (n2, row) in sorted(self.slot.items(), key=lambda kv: kv[1]):
                if n2 != log2n:
                    continue
                keys_a.append(synth.key(seed, r, l, 0, 0))
                keys_b.append(synth.key(seed, r, l, 0, 1))
                qs.append(prm.q[l])
            for s0 in range(0, S, chunk):
                s1 = min(S, s0 + chunk)
                synth.uniform_mod_device(keys_a[s0:s1], N, qs[s0:s1], a[s0:s1])
                synth.uniform_mod_device(keys_b[s0:s1], N, qs[s0:s1], b[s0:s1])
            self.a[log2n], self.b[log2n] = a, b
            self.c[log2n] = torch.empty_like(a)
        self.jobs = []
        for (r, l), (log2n, row) in sorted(self.slot.items()):
            prm = self.tables.get(log2n, 0)
            self.jobs.append(lib.make_job(log2n, 1, prm.q[l], prm.psi_br[l], prm.psi_inv_br[l],
                                          self.a[log2n][row], self.b[log2n][row], self.c[log2n][row]))

    @property
    def products(self) -> int:
        return len(self.slot)

    def modulus(self, r, l):
        log2n, _ = self.slot[(r, l)]
        return self.tables.get(log2n, 0).q[l]

    def modulus_of_limb(self, log2n, l):
        """Limb l's modulus for size 2^log2n (the l-th largest prime q = 1 mod 2N)."""
        return self.tables.get(log2n, 0).q[l]

    def host_operands(self, r, l):
        """The same (a, b) drawn again on the host."""
        log2n, _ = self.slot[(r, l)]
        q = self.modulus(r, l)
        N = 1 << log2n
        return (synth.uniform_mod(synth.key(self.seed, r, l, 0, 0), N, q),
                synth.uniform_mod(synth.key(self.seed, r, l, 0, 1), N, q))

    def device_row(self, which, r, l):
        log2n, row = self.slot[(r, l)]
        return getattr(self, which)[log2n][row]

    def request_limbs(self, r):
        """(a, b, c) device views of request r's limbs, or None when its rows
        are not contiguous in their N block."""
        log2n, L = self.requests[r]
        first = self.slot[(r, 0)][1]
        return (self.a[log2n][first:first + L], self.b[log2n][first:first + L], self.c[log2n][first:first + L])
