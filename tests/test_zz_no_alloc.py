"""pm_polymul_noalloc: the product with its workspace in the library's fixed
per-GPU scratch array, called through the C ABI and compared word for word
with pm_polymul (caller workspace) on the same inputs, and sampled against
the oracle. Tolerance zero."""
import numpy as np
import pytest

from gpu_helpers import device_tables, first_mismatch, operands, oracle_polymul

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


def _case(L, N, limbs, polys, seed):
    import torch
    qs = L.pm_ntt_primes(N, limbs)
    fw, iv, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, seed=seed)
    dev = torch.device("cuda:0")
    return qs, fw, iv, dfw, div, a, b, L.to_device(a, dev), L.to_device(b, dev)


def _reference(L, N, limbs, polys, qs, dfw, div, da, db):
    import torch
    dc = torch.empty_like(da)
    nb = L.pm_polymul_workspace_bytes(N, limbs, polys)
    ws = torch.empty(max(nb // 8, 1), dtype=torch.int64, device=da.device)
    L.pm_polymul(da, db, dc, N, limbs, polys, qs, dfw, div, ws)
    return dc


def _check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, "%s: %s" % (what, msg)


# (N, limbs, polys): the first needs exactly the 64 MiB scratch (128 products
# of 2^16, the software-pipelined form); the second is smaller and runs the
# three-pass form over the scratch left by the first; then a small-batch plan,
# and a single-pass size that needs no workspace.
SEQUENCES = [
    [(1 << 16, 4, 32), (1 << 14, 3, 5)],
    [(1 << 17, 2, 32), (1 << 15, 1, 3)],
    [(1 << 13, 5, 7), (1 << 10, 2, 2)],
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=lambda s: "->".join("%dx%dx%d" % t for t in s))
def test_noalloc_equals_polymul_two_calls(L, seq):
    import torch
    cases = []
    for k, (N, limbs, polys) in enumerate(seq):
        print("[no_alloc] N=%d limbs=%d polys=%d" % (N, limbs, polys), flush=True)
        qs, fw, iv, dfw, div, a, b, da, db = _case(L, N, limbs, polys, seed=9100 + k)
        assert L.pm_polymul_workspace_bytes(N, limbs, polys) <= L.PM_NOALLOC_SCRATCH_BYTES
        cases.append((N, limbs, polys, qs, fw, iv, dfw, div, a, b, da, db))
    # the two no-alloc calls back to back on one stream, then the references
    outs = []
    for (N, limbs, polys, qs, fw, iv, dfw, div, a, b, da, db) in cases:
        dc = torch.full_like(da, -1)
        L.pm_polymul_noalloc(da, db, dc, N, limbs, polys, qs, dfw, div)
        outs.append(dc)
    torch.cuda.synchronize()
    for (N, limbs, polys, qs, fw, iv, dfw, div, a, b, da, db), dc in zip(cases, outs):
        ref = _reference(L, N, limbs, polys, qs, dfw, div, da, db)
        torch.cuda.synchronize()
        got = L.to_host(dc).reshape(a.shape)
        _check(got, L.to_host(ref).reshape(a.shape), "noalloc vs pm_polymul, N=%d %dx%d" % (N, limbs, polys))
        # a sampled product against the oracle as well
        l, p = limbs - 1, polys - 1
        want = oracle_polymul(a[l:l + 1, p:p + 1], b[l:l + 1, p:p + 1], qs[l:l + 1], N, fw[l:l + 1], iv[l:l + 1])
        _check(got[l:l + 1, p:p + 1], want, "noalloc vs oracle, N=%d limb %d pair %d" % (N, l, p))


def test_noalloc_aliasing_and_square(L):
    import torch
    N, limbs, polys = 1 << 16, 2, 8
    qs, fw, iv, dfw, div, a, b, da, db = _case(L, N, limbs, polys, seed=9200)
    ref = _reference(L, N, limbs, polys, qs, dfw, div, da, db)
    sq = _reference(L, N, limbs, polys, qs, dfw, div, da, da)
    x = da.clone()
    L.pm_polymul_noalloc(x, db, x, N, limbs, polys, qs, dfw, div)           # c aliases a
    y = db.clone()
    L.pm_polymul_noalloc(da, y, y, N, limbs, polys, qs, dfw, div)           # c aliases b
    z = torch.empty_like(da)
    L.pm_polymul_noalloc(da, da, z, N, limbs, polys, qs, dfw, div)          # a = b
    torch.cuda.synchronize()
    r = L.to_host(ref)
    _check(L.to_host(x), r, "c aliases a")
    _check(L.to_host(y), r, "c aliases b")
    _check(L.to_host(z), L.to_host(sq), "a = b")


def test_noalloc_rejects_batches_above_the_scratch(L):
    import torch
    N, limbs, polys = 1 << 16, 4, 33            # 132 products: 66 MiB of workspace
    assert L.pm_polymul_workspace_bytes(N, limbs, polys) > L.PM_NOALLOC_SCRATCH_BYTES
    qs = L.pm_ntt_primes(N, limbs)
    small = torch.zeros(8, dtype=torch.int64, device="cuda:0")   # never read: rejected before any launch
    with pytest.raises(L.PMError) as ei:
        L.pm_polymul_noalloc(small, small, small, N, limbs, polys, qs, small, small)
    assert ei.value.code == L.PM_EINVAL
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
