"""The batched mixed workload at full size (512 requests, N uniform on
2^12..2^17, 1..48 limbs each: ~12.5k limb-products) in one plan launch,
checked on sampled products against the oracle; plus the device-side input
generator against the host one."""
import numpy as np
import pytest

import oracle
from gpu_helpers import first_mismatch, tuned
from paper_2209_01290_amd import synth, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


def test_device_generator_matches_host(L):
    import torch
    keys = [synth.key(3, r, l, 0, o) for r in range(4) for l in range(2) for o in range(2)]
    qs = [0x0FFFFFFFFFFFC001, 97, 12289, (1 << 62) - 57, 2**35 - 31, 3, 65537, 2**30 + 3] * 2
    out = torch.empty((16, 4099), dtype=torch.int64, device="cuda")
    synth.uniform_mod_device(keys, 4099, qs, out)
    host = out.cpu().numpy().view(np.uint64)
    for s in range(16):
        assert np.array_equal(host[s], synth.uniform_mod(keys[s], 4099, qs[s])), s


def test_config4_mixed_full_size(L):
    """All 13,096 limb-products of the 512-request batch, from one plan launch
    (the software-pipelined job table the benchmark times), each compared word
    for word with the oracle; the one-shot form in both the pipelined and the
    three-pass layout gives the same words; the device generator matches the
    host one on sampled rows."""
    import torch
    from gpu_helpers import oracle_parallel
    reqs = workloads.mixed_requests(synth.SEED_BASE + 4)
    assert len(reqs) == 512 and {n for n, _ in reqs} == set(range(12, 18))
    mb = workloads.MixedBatch(reqs, synth.SEED_BASE + 4, torch.device("cuda"))
    assert mb.products == 13096
    with tuned(L):                       # plans read the tuned table at creation, as in the benchmark
        plan = L.pm_plan_create(mb.jobs)
    try:
        L.pm_plan_launch(plan)
        torch.cuda.synchronize()
    finally:
        L.pm_plan_destroy(plan)
    plan_out = {n: c.clone() for n, c in mb.c.items()}
    # the one-shot form, pipelined (default) and three-pass, equals the plan for every product
    for chunks in (-1, 0):
        for c in mb.c.values():
            c.zero_()
        L.pm_tune_set_jobs_pipeline(chunks)
        try:
            nbytes = L.pm_polymul_jobs_workspace_bytes(mb.jobs)
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
            L.pm_polymul_jobs(mb.jobs, ws)
            torch.cuda.synchronize()
            del ws
        finally:
            L.pm_tune_set_jobs_pipeline(-1)
        for n in mb.c:
            assert torch.equal(mb.c[n], plan_out[n]), "N=2^%d: one-shot (chunks %d) differs from the plan" % (n, chunks)
    # sampled rows: the device generator equals the host one
    rng = np.random.default_rng(4)
    by_n = {}
    for r, (n, Lr) in enumerate(reqs):
        by_n.setdefault(n, []).append((r, Lr))
    for n, lst in sorted(by_n.items()):
        r, Lr = lst[int(rng.integers(len(lst)))]
        for l in (0, Lr - 1):
            a, b = mb.host_operands(r, l)
            assert np.array_equal(L.to_host(mb.device_row("a", r, l)), a), (r, l)
            assert np.array_equal(L.to_host(mb.device_row("b", r, l)), b), (r, l)
    # every product against the oracle, one size at a time, over the host's cores
    o = oracle.default()
    checked = 0
    for log2n in sorted(plan_out):
        N = 1 << log2n
        A, B, C = (L.to_host(t).reshape(-1, N) for t in (mb.a[log2n], mb.b[log2n], plan_out[log2n]))
        items = sorted((row, r, l) for (r, l), (n2, row) in mb.slot.items() if n2 == log2n)
        limbs = sorted({l for _, _, l in items})
        tabs = dict(zip(limbs, oracle_parallel(lambda l: o.psi_tables(mb.modulus_of_limb(log2n, l), N), limbs)))

        def check(item):
            row, r, l = item
            fw, iv = tabs[l]
            want = o.polymul_ntt(A[row], B[row], mb.modulus_of_limb(log2n, l), fw, iv)
            return None if np.array_equal(C[row], want) else "request %d limb %d (N=2^%d): %s" % (
                r, l, log2n, first_mismatch(C[row], want))

        bad = [m for m in oracle_parallel(check, items) if m]
        assert not bad, "%d products differ from the oracle; first: %s" % (len(bad), bad[0])
        checked += len(items)
        del A, B, C
    assert checked == 13096
