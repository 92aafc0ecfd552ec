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
    import torch
    reqs = workloads.mixed_requests(synth.SEED_BASE + 4)
    assert len(reqs) == 512 and {n for n, _ in reqs} == set(range(12, 18))
    mb = workloads.MixedBatch(reqs, synth.SEED_BASE + 4, torch.device("cuda"))
    with tuned(L):                       # plans read the tuned table at creation, as in the benchmark
        plan = L.pm_plan_create(mb.jobs)
    try:
        L.pm_plan_launch(plan)
        torch.cuda.synchronize()
    finally:
        L.pm_plan_destroy(plan)
    o = oracle.default()
    rng = np.random.default_rng(4)
    by_n = {}
    for r, (n, Lr) in enumerate(reqs):
        by_n.setdefault(n, []).append((r, Lr))
    samples = []
    for n, lst in sorted(by_n.items()):
        r, Lr = lst[int(rng.integers(len(lst)))]
        samples += [(r, 0), (r, Lr - 1)]
    for r, l in samples:
        log2n, _ = mb.slot[(r, l)]
        N = 1 << log2n
        q = mb.modulus(r, l)
        a, b = mb.host_operands(r, l)
        assert np.array_equal(L.to_host(mb.device_row("a", r, l)), a)
        fw, iv = o.psi_tables(q, N)
        want = o.polymul_ntt(a, b, q, fw, iv)
        msg = first_mismatch(L.to_host(mb.device_row("c", r, l)), want)
        assert msg is None, "request %d limb %d (N=2^%d): %s" % (r, l, log2n, msg)
    # the one-shot form gives the same words for every product
    plan_out = {n: c.clone() for n, c in mb.c.items()}
    for c in mb.c.values():
        c.zero_()
    nbytes = L.pm_polymul_jobs_workspace_bytes(mb.jobs)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
    L.pm_polymul_jobs(mb.jobs, ws)
    torch.cuda.synchronize()
    for n in mb.c:
        assert torch.equal(mb.c[n], plan_out[n]), n
