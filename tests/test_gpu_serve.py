"""The serving loop on the GPU: results are identical alone and in the mix
(tolerance 0), match the oracle on sampled limbs, and every request finishes
under queueing pressure."""
import numpy as np
import pytest

import oracle
from gpu_helpers import first_mismatch, tuned
from paper_2209_01290_amd import serve, synth, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return serve.GpuExecutor(4 << 30, streams=3, pool=2)


def test_alone_equals_mix_and_oracle(ex):
    trace = workloads.serving_requests(serve.SEED + 1, 240, 10000.0)
    saved = {}
    sample = set(range(0, 240, 12)) | {239}

    def keep(r, executor):
        if r.rid in sample:
            saved[r.rid] = (r, executor.output(r).cpu())

    eng = serve.Engine(ex, ex.budget(), streams=3)
    st = eng.run(trace, on_complete=keep)
    assert st["completed"] == 240 and st["rejected"] == 0
    assert st["max_inflight_batches"] >= 2
    for rid, (r, mix) in sorted(saved.items()):
        alone = ex.run_alone(r).cpu()
        assert np.array_equal(alone.numpy(), mix.numpy()), "request %d differs alone vs in the mix" % rid
    o = oracle.default()
    for rid in sorted(saved)[:2]:
        r, mix = saved[rid]
        N = 1 << r.log2n
        prm = ex.tables.get(r.log2n, 0)
        p = r.rid % ex.pool
        for l in [0, r.limbs - 1]:
            q = prm.q[l]
            a = synth.uniform_mod(synth.key(ex.seed, p, l, 0, 0), N, q)
            b = synth.uniform_mod(synth.key(ex.seed, p, l, 0, 1), N, q)
            fw, iv = o.psi_tables(q, N)
            msg = first_mismatch(mix[l].numpy().view(np.uint64), o.polymul_ntt(a, b, q, fw, iv))
            assert msg is None, "request %d limb %d: %s" % (rid, l, msg)


def test_small_budget_queues_and_completes(ex):
    trace = workloads.serving_requests(serve.SEED + 2, 120, 50000.0)
    one = max(serve.request_bytes(n, L) for _, n, L in trace) + serve.BATCH_WS_SLACK
    eng = serve.Engine(ex, 2 * one, streams=3)
    st = eng.run(trace)
    assert st["completed"] == 120 and st["max_queue"] > 1
    assert st["arena_peak_bytes"] <= 2 * one


def test_single_request_batches_match_jobs_path(ex):
    """Below saturation most batches hold one request, which runs as one
    pm_polymul (small-batch plans installed); every result equals the same
    request through pm_polymul_jobs alone."""
    from paper_2209_01290_amd import lib
    trace = workloads.serving_requests(serve.SEED + 3, 40, 300.0)
    outs = {}

    def keep(r, executor):
        outs[r.rid] = (r, executor.output(r).cpu())

    with tuned(lib):
        st = serve.Engine(ex, ex.budget(), streams=3).run(trace, on_complete=keep)
    # 40 requests in B batches leave at least 2B - 40 batches of one request
    assert st["completed"] == 40 and st["batches"] >= 24, st
    for rid, (r, mix) in sorted(outs.items()):
        alone = ex.run_alone(r).cpu()
        assert np.array_equal(alone.numpy(), mix.numpy()), "request %d: single-request path vs jobs path" % rid
