"""PM_VALIDATE=1: the entry points reject non-canonical inputs and tables
whose psi fails psi^N = q - 1 (PM_EINVAL, before any output is written),
and accept valid calls with unchanged results."""
import numpy as np
import pytest

from gpu_helpers import first_mismatch, operands, oracle_polymul, oracle_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


@pytest.fixture
def validate(monkeypatch):
    monkeypatch.setenv("PM_VALIDATE", "1")
    yield


def _sync():
    import torch
    torch.cuda.synchronize()


def _setup(L, log2n=12, limbs=3, polys=2, request=2300):
    N = 1 << log2n
    qs = L.pm_ntt_primes(N, limbs)
    prm = L.Params(N, limbs, primes=qs)
    a, b = operands(N, qs, polys, request=request)
    return N, qs, prm, a, b


def _ws(L, N, limbs, polys):
    import torch
    n = L.pm_polymul_workspace_bytes(N, limbs, polys)
    return torch.empty(max(n // 8, 1), dtype=torch.int64, device="cuda")


def _expect_einval(L, fn, text):
    with pytest.raises(L.PMError) as ei:
        fn()
    assert ei.value.code == L.PM_EINVAL, str(ei.value)
    assert text in str(ei.value), str(ei.value)


@pytest.mark.parametrize("log2n", [6, 12, 16])
def test_valid_calls_pass(L, validate, log2n):
    import torch
    N, qs, prm, a, b = _setup(L, log2n)
    limbs, polys = a.shape[0], a.shape[1]
    da, db = L.to_device(a), L.to_device(b)
    dc = torch.empty_like(da)
    L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    x = da.clone()
    L.pm_ntt_fwd(x, N, limbs, polys, qs, prm.psi_br)
    L.pm_ntt_inv(x, N, limbs, polys, qs, prm.psi_inv_br)
    _sync()
    fw, iv = oracle_tables(qs, N)
    assert first_mismatch(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw, iv)) is None
    assert first_mismatch(L.to_host(x).reshape(a.shape), a) is None


def test_non_canonical_input_rejected(L, validate):
    import torch
    N, qs, prm, a, b = _setup(L)
    limbs, polys = a.shape[0], a.shape[1]
    bad = a.copy()
    bad[1, 1, 77] = qs[1]
    da, db = L.to_device(bad), L.to_device(b)
    dc = torch.zeros_like(da)
    ws = _ws(L, N, limbs, polys)
    _expect_einval(L, lambda: L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws),
                   "a: limb 1 holds a word >= q")
    _expect_einval(L, lambda: L.pm_polymul(db, da, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws),
                   "b: limb 1")
    _expect_einval(L, lambda: L.pm_polymul_fused(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws),
                   "limb 1")
    _expect_einval(L, lambda: L.pm_ntt_fwd(da, N, limbs, polys, qs, prm.psi_br), "x: limb 1")
    _expect_einval(L, lambda: L.pm_ntt_inv(da, N, limbs, polys, qs, prm.psi_inv_br), "x: limb 1")
    _expect_einval(L, lambda: L.pm_polymul_stagewise(
        da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br,
        torch.empty(L.pm_polymul_stagewise_workspace_bytes(N, limbs, polys) // 8, dtype=torch.int64,
                    device="cuda")), "limb 1")
    _sync()
    assert not dc.any().item(), "output written despite the error"
    assert np.array_equal(L.to_host(da).reshape(a.shape), bad), "input modified despite the error"
    # the elementwise product: one word equal to q
    x = L.to_device(np.array([1, 2, qs[0]], dtype=np.uint64))
    y = L.to_device(np.array([3, 4, 5], dtype=np.uint64))
    z = torch.empty_like(x)
    _expect_einval(L, lambda: L.pm_barrett_mulmod(x, y, z, qs[0]), "a: limb 0")


def test_bad_tables_rejected(L, validate):
    import torch
    N, qs, prm, a, b = _setup(L)
    limbs, polys = a.shape[0], a.shape[1]
    da, db = L.to_device(a), L.to_device(b)
    dc = torch.zeros_like(da)
    ws = _ws(L, N, limbs, polys)
    bad_f = prm.psi_br.clone()
    bad_f[2, N // 2] = 1                   # 1^N = 1 != q - 1
    _expect_einval(L, lambda: L.pm_ntt_fwd(da, N, limbs, polys, qs, bad_f), "psi_br: limb 2")
    _expect_einval(L, lambda: L.pm_polymul(da, db, dc, N, limbs, polys, qs, bad_f, prm.psi_inv_br, ws),
                   "psi_br: limb 2")
    bad_i = prm.psi_inv_br.clone()
    bad_i[0, N // 2] = 0
    _expect_einval(L, lambda: L.pm_ntt_inv(da, N, limbs, polys, qs, bad_i), "psi_inv_br: limb 0")
    # a table built for another modulus
    other = L.Params(N, limbs, primes=L.pm_ntt_primes(N, limbs + 1)[1:])
    _expect_einval(L, lambda: L.pm_polymul(da, db, dc, N, limbs, polys, qs, other.psi_br, prm.psi_inv_br, ws),
                   "psi_br")
    _sync()
    assert not dc.any().item()


def test_u32_and_interleaved(L, validate):
    import torch
    N, limbs, polys = 1 << 10, 2, 2
    qs = L.pm_ntt_primes(N, limbs, 30)
    p32 = L.Params32(N, limbs, primes=qs)
    a, b = operands(N, qs, polys, request=2400)
    bad = a.copy()
    bad[0, 1, 3] = qs[0] + 5
    da, db = L.to_device32(bad), L.to_device32(b)
    dc = torch.zeros_like(da)
    _expect_einval(L, lambda: L.pm_polymul_u32(da, db, dc, N, limbs, polys, qs, p32.psi_br, p32.psi_inv_br),
                   "a: limb 0")
    ok = L.to_device32(a)
    L.pm_polymul_u32(ok, db, dc, N, limbs, polys, qs, p32.psi_br, p32.psi_inv_br)
    _sync()
    qs64 = L.pm_ntt_primes(N, limbs)
    p64 = L.Params(N, limbs, primes=qs64)
    a64, b64 = operands(N, qs64, polys, request=2401)
    a64[1, 0, 9] = qs64[1]
    x = L.to_device(np.ascontiguousarray(np.transpose(a64, (0, 2, 1))))
    _expect_einval(L, lambda: L.pm_ntt_fwd_il(x, N, limbs, polys, qs64, p64.psi_br), "x: limb 1")


def test_jobs_and_plans(L, validate):
    import torch
    N, qs, prm, a, b = _setup(L, log2n=13, limbs=2, polys=1)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch.zeros_like(da)
    jobs = [L.make_job(13, 1, qs[l], prm.psi_br[l], prm.psi_inv_br[l], da[l], db[l], dc[l]) for l in range(2)]
    plan = L.pm_plan_create(jobs)
    try:
        L.pm_plan_launch(plan)
        _sync()
        fw, iv = oracle_tables(qs, N)
        assert first_mismatch(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw, iv)) is None
        bad = a.copy()
        bad[1, 0, 0] = qs[1]
        da.copy_(L.to_device(bad))
        _expect_einval(L, lambda: L.pm_plan_launch(plan), "job 1: a")
    finally:
        L.pm_plan_destroy(plan)
    bad_t = prm.psi_inv_br.clone()
    bad_t[0, N // 2] = 0
    jobs = [L.make_job(13, 1, qs[0], prm.psi_br[0], bad_t[0], db[0], db[0], dc[0])]
    _expect_einval(L, lambda: L.pm_plan_create(jobs), "job 0: psi_inv_br")


def test_without_validate_non_canonical_is_accepted(L, monkeypatch):
    import torch
    monkeypatch.delenv("PM_VALIDATE", raising=False)
    N, qs, prm, a, b = _setup(L)
    limbs, polys = a.shape[0], a.shape[1]
    bad = a.copy()
    bad[0, 0, 0] = qs[0]
    da, db = L.to_device(bad), L.to_device(b)
    dc = torch.empty_like(da)
    L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    _sync()
