"""Shared helpers for the GPU parity tests (operands, tables, oracle checks)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2209_01290_amd import synth

SEED = synth.SEED_BASE


def operands(N, qs, polys, seed=SEED, request=0):
    return synth.operands(seed, qs, polys, N, request=request)


def oracle_tables(qs, N):
    o = oracle.default()
    fw = np.empty((len(qs), N), np.uint64)
    iv = np.empty((len(qs), N), np.uint64)
    for l, q in enumerate(qs):
        fw[l], iv[l] = o.psi_tables(q, N)
    return fw, iv


def device_tables(qs, N):
    """Tables built by the library's own host helper, uploaded."""
    from paper_2209_01290_amd import lib
    fw = np.empty((len(qs), N), np.uint64)
    iv = np.empty((len(qs), N), np.uint64)
    for l, q in enumerate(qs):
        fw[l], iv[l] = lib.pm_make_tables(q, N)
    return fw, iv, lib.to_device(fw), lib.to_device(iv)


def oracle_polymul(a, b, qs, N, fw, iv):
    o = oracle.default()
    L, P = a.shape[0], a.shape[1]
    c = np.empty_like(a)
    for l in range(L):
        for p in range(P):
            c[l, p] = o.polymul_ntt(a[l, p], b[l, p], qs[l], fw[l], iv[l])
    return c


def oracle_ntt_fwd(x, qs, fw):
    o = oracle.default()
    y = np.empty_like(x)
    for l in range(x.shape[0]):
        for p in range(x.shape[1]):
            y[l, p] = o.ntt_fwd(x[l, p], qs[l], fw[l])
    return y


def oracle_ntt_inv(x, qs, iv):
    o = oracle.default()
    y = np.empty_like(x)
    for l in range(x.shape[0]):
        for p in range(x.shape[1]):
            y[l, p] = o.ntt_inv(x[l, p], qs[l], iv[l])
    return y


def first_mismatch(got, want):
    bad = np.nonzero(got.reshape(-1) != want.reshape(-1))[0]
    if bad.size == 0:
        return None
    i = int(bad[0])
    return "%d mismatches, first at flat index %d: got %d want %d" % (
        bad.size, i, int(got.reshape(-1)[i]), int(want.reshape(-1)[i]))


class tuned:
    """Context manager: the packaged tuning database installed (the plans
    bench.py runs), every plan table back to the library defaults on exit."""

    def __init__(self, L):
        self.L = L

    def __enter__(self):
        self.L.apply_tune_db()
        return self

    def __exit__(self, *exc):
        L = self.L
        for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
            for n in range(1, 18):
                L.pm_tune_set(op, n, 0)
                L.pm_tune_set_small(op, n, 0, 0)
                L.pm_tune_set_small_limit(op, n, 0)
        L.pm_tune_set_small_batch(0)
        L.pm_tune_set_pipeline(-1)
        for logr in (3, 4, 5):
            L.pm_tune_set_pipeline_rows(logr, 0)
        L.pm_tune_set_jobs_pipeline(-1)
        return False


def host_threads():
    """Worker threads for oracle checks: the CPUs this process may use, at most 16."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_parallel(fn, items, threads=None):
    """[fn(item) for item in items] over a thread pool (the oracle's ctypes
    calls release the interpreter lock, so the C work runs in parallel)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(threads or host_threads()) as ex:
        return list(ex.map(fn, items))
