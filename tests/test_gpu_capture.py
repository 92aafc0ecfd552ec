"""The library under HIP-graph capture and under concurrent host threads.

Capture: pm_polymul and pm_ntt_fwd (throughput, small-batch and
software-pipelined plans) are captured into one graph; the graph is replayed several times with eager work
and synchronisations between replays, and every replay must reproduce the
eager results bit for bit (the library records no memset nodes).
Threads: four host threads issue products on their own streams at once;
every result must equal the oracle's."""
import threading

import numpy as np
import pytest

from gpu_helpers import first_mismatch, operands, oracle_ntt_fwd, oracle_polymul, oracle_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


def _eq(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, "%s: %s" % (what, msg)


@pytest.mark.parametrize("small", [False, True, "pipelined"], ids=["throughput", "small", "pipelined"])
@pytest.mark.parametrize("log2n", [10, 14, 16])
def test_graph_capture_replays(L, log2n, small):
    import torch
    if small == "pipelined":
        log2n = {10: 15, 14: 16, 16: 17}[log2n]     # the pipelined plan needs N = 2^15..2^17
    N, limbs, polys = 1 << log2n, 2, 2
    qs = L.pm_ntt_primes(N, limbs)
    prm = L.Params(N, limbs, primes=qs)
    a, b = operands(N, qs, polys, request=2100 + log2n)
    fw_o, iv_o = oracle_tables(qs, N)
    want_mul = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    want_fwd = oracle_ntt_fwd(a, qs, fw_o)
    try:
        if small == "pipelined":
            L.pm_tune_set_pipeline(2)
        elif small:
            for op in (L.OP_NTT_FWD, L.OP_POLYMUL):
                L.pm_tune_set_small(op, log2n, min(log2n, 11) if log2n > 12 else log2n, 4)
            L.pm_tune_set_small_batch(1 << 22)
        da, db = L.to_device(a), L.to_device(b)
        dc = torch.empty_like(da)
        x = torch.empty_like(da)
        nbytes = L.pm_polymul_workspace_bytes(N, limbs, polys)
        ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device="cuda")

        def work():
            L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws)
            x.copy_(da)
            L.pm_ntt_fwd(x, N, limbs, polys, qs, prm.psi_br)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            work()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        _eq(L.to_host(dc).reshape(a.shape), want_mul, "eager polymul")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            work()
        for rep in range(4):
            dc.zero_()
            x.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            _eq(L.to_host(dc).reshape(a.shape), want_mul, "replay %d polymul" % rep)
            _eq(L.to_host(x).reshape(a.shape), want_fwd, "replay %d ntt_fwd" % rep)
            # eager work between replays
            L.pm_ntt_fwd(x, N, limbs, polys, qs, prm.psi_br)
            torch.cuda.synchronize()
        del g
        if small == "pipelined":           # the captured launches were the pipelined ones
            counts = {}
            L.pm_prof_enable(True)
            try:
                L.pm_prof_read()
                L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws)
                torch.cuda.synchronize()
                counts = {k: n for k, (n, _ms) in L.pm_prof_read().items()}
            finally:
                L.pm_prof_enable(False)
            assert counts.get("pipe_mul_c12", 0) == 4, counts
    finally:
        L.pm_tune_set_pipeline(-1)
        for op in (L.OP_NTT_FWD, L.OP_POLYMUL):
            L.pm_tune_set_small(op, log2n, 0, 0)
        L.pm_tune_set_small_batch(0)


def test_concurrent_host_threads(L):
    import torch
    N, limbs, polys = 1 << 14, 3, 2
    qs = L.pm_ntt_primes(N, limbs)
    prm = L.Params(N, limbs, primes=qs)
    fw_o, iv_o = oracle_tables(qs, N)
    nthreads = 4
    inputs = [operands(N, qs, polys, request=2200 + t) for t in range(nthreads)]
    results, errors = [None] * nthreads, []

    def run(t):
        try:
            a, b = inputs[t]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                da, db = L.to_device(a), L.to_device(b)
                dc = torch.empty_like(da)
                nbytes = L.pm_polymul_workspace_bytes(N, limbs, polys)
                ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device="cuda")
                for _ in range(5):
                    L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws, stream=s)
            s.synchronize()
            results[t] = L.to_host(dc).reshape(a.shape)
        except Exception as e:      # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=run, args=(t,)) for t in range(nthreads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for t in range(nthreads):
        a, b = inputs[t]
        _eq(results[t], oracle_polymul(a, b, qs, N, fw_o, iv_o), "thread %d" % t)
