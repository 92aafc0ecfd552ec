"""Small-batch pass plans (4 words per thread in both passes, shorter rows):
bit-exact parity with the CPU oracle for every valid (N, row length) under the
4-word geometry, on 64- and 32-bit words, and the threshold that selects them
(checked through the names of the kernels the library launched)."""
import functools

import numpy as np
import pytest

from gpu_helpers import first_mismatch, operands, oracle_ntt_fwd, oracle_ntt_inv, oracle_polymul, oracle_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


@pytest.fixture
def small(L):
    """Clears every small-batch plan and the threshold after the test."""
    yield
    for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
        for n in range(1, 18):
            L.pm_tune_set_small(op, n, 0, 0)
            L.pm_tune_set_small_limit(op, n, 0)
    L.pm_tune_set_small_batch(0)


def _sync():
    import torch
    torch.cuda.synchronize()


def _eq(got, want, what):
    msg = first_mismatch(np.asarray(got, dtype=np.uint64), np.asarray(want, dtype=np.uint64))
    assert msg is None, "%s: %s" % (what, msg)


def small_plans():
    """Every (log2 N, log2 C) of the 4-word geometry: rows of 2^5..2^12 words,
    column passes of 2^2..2^7 rows (four words per thread) or of 2 rows with
    one thread per column (>= 256 columns)."""
    out = []
    for log2n in range(5, 18):
        for logc in range(5, min(log2n, 12) + 1):
            logr = log2n - logc
            if logr > 7 or (logr == 1 and logc < 8):
                continue
            out.append((log2n, logc))
    return out


@functools.lru_cache(maxsize=None)
def _case64(log2n):
    """Operands and oracle results for N = 2^log2n, two 60-bit limbs, two pairs."""
    N, limbs, polys = 1 << log2n, 2, 2
    from paper_2209_01290_amd import lib
    qs = lib.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    a, b = operands(N, qs, polys, request=1500 + log2n)
    return (qs, a, b, oracle_ntt_fwd(a, qs, fw_o), oracle_ntt_inv(a, qs, iv_o),
            oracle_polymul(a, b, qs, N, fw_o, iv_o), oracle_polymul(a, a, qs, N, fw_o, iv_o))


@functools.lru_cache(maxsize=None)
def _case32(log2n):
    """Operands and oracle results for N = 2^log2n, two 30-bit limbs, two pairs."""
    N, limbs, polys = 1 << log2n, 2, 2
    from paper_2209_01290_amd import lib
    qs = lib.pm_ntt_primes(N, limbs, 30)
    fw_o, iv_o = oracle_tables(qs, N)
    a, b = operands(N, qs, polys, request=1600 + log2n)
    return (qs, a, b, oracle_ntt_fwd(a, qs, fw_o), oracle_ntt_inv(a, qs, iv_o),
            oracle_polymul(a, b, qs, N, fw_o, iv_o))


def _col_kernel(log2n, logc, inv=False):
    logr = log2n - logc
    if logr == 0:
        return None
    return ("colq" if logr >= 2 else "col") + ("_inv_r%d" if inv else "_fwd_r%d") % logr


def _install(L, log2n, logc, wpt=4):
    for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
        L.pm_tune_set_small(op, log2n, logc, wpt)
    L.pm_tune_set_small_batch(1 << 22)


def _ws(L, N, limbs, polys, u32=False):
    import torch
    n = (L.pm_polymul_u32_workspace_bytes if u32 else L.pm_polymul_workspace_bytes)(N, limbs, polys)
    return torch.empty(max(n // 8, 1), dtype=torch.int64, device="cuda") if n else None


@pytest.mark.parametrize("log2n,logc", small_plans(), ids=lambda v: str(v))
def test_small_plan_u64(L, small, log2n, logc):
    import torch
    N, limbs, polys = 1 << log2n, 2, 2
    _install(L, log2n, logc)
    qs, a, b, want_fwd, want_inv, want, want_sq = _case64(log2n)
    prm = L.Params(N, limbs, primes=qs)
    L.pm_prof_read(reset=True)
    L.pm_prof_enable(True)
    try:
        x = L.to_device(a)
        L.pm_ntt_fwd(x, N, limbs, polys, qs, prm.psi_br)
        _sync()
        _eq(L.to_host(x).reshape(a.shape), want_fwd, "fwd N=%d c=%d" % (N, logc))
        y = L.to_device(a)
        L.pm_ntt_inv(y, N, limbs, polys, qs, prm.psi_inv_br)
        _sync()
        _eq(L.to_host(y).reshape(a.shape), want_inv, "inv N=%d c=%d" % (N, logc))
        da, db = L.to_device(a), L.to_device(b)
        dc = torch.empty_like(da)
        L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
        _sync()
        _eq(L.to_host(dc).reshape(a.shape), want, "polymul N=%d c=%d" % (N, logc))
        # a = b (the 4-word geometry runs the product with b = a) and c = a
        L.pm_polymul(da, da, da, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, None)
        _sync()
        _eq(L.to_host(da).reshape(a.shape), want_sq, "square N=%d c=%d" % (N, logc))
        # the fused product keeps the 16-word rows under the same split
        df = torch.empty_like(db)
        L.pm_polymul_fused(L.to_device(a), db, df, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br,
                           _ws(L, N, limbs, polys))
        _sync()
        _eq(L.to_host(df).reshape(a.shape), want, "fused N=%d c=%d" % (N, logc))
    finally:
        L.pm_prof_enable(False)
    names = L.pm_prof_read(reset=True)
    assert "row_fwd_c%ds" % logc in names and "row_mul_c%ds" % logc in names, sorted(names)
    assert "row_fmul_c%d" % logc in names
    if log2n > logc:
        assert _col_kernel(log2n, logc) in names and _col_kernel(log2n, logc, True) in names, sorted(names)


@pytest.mark.parametrize("log2n,logc", [p for p in small_plans() if p[0] in (10, 12, 14, 16, 17)],
                         ids=lambda v: str(v))
def test_small_plan_u32(L, small, log2n, logc):
    import torch
    N, limbs, polys = 1 << log2n, 2, 2
    _install(L, log2n, logc)
    qs, a, b, want_fwd, want_inv, want = _case32(log2n)
    prm = L.Params32(N, limbs, primes=qs)
    x = L.to_device32(a)
    L.pm_ntt_fwd_u32(x, N, limbs, polys, qs, prm.psi_br)
    _sync()
    _eq(L.to_host32(x).reshape(a.shape), want_fwd, "fwd32 N=%d c=%d" % (N, logc))
    L.pm_ntt_inv_u32(x, N, limbs, polys, qs, prm.psi_inv_br)
    _sync()
    _eq(L.to_host32(x).reshape(a.shape), a, "roundtrip32 N=%d c=%d" % (N, logc))
    y = L.to_device32(a)
    L.pm_ntt_inv_u32(y, N, limbs, polys, qs, prm.psi_inv_br)
    _sync()
    _eq(L.to_host32(y).reshape(a.shape), want_inv, "inv32 N=%d c=%d" % (N, logc))
    da, db = L.to_device32(a), L.to_device32(b)
    dc = torch.empty_like(da)
    L.pm_polymul_u32(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys, True))
    _sync()
    _eq(L.to_host32(dc).reshape(a.shape), want, "polymul32 N=%d c=%d" % (N, logc))
    # the fused product (16-word rows) over the same column pass
    df = torch.empty_like(da)
    L.pm_polymul_fused_u32(da, db, df, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br,
                           _ws(L, N, limbs, polys, True))
    _sync()
    _eq(L.to_host32(df).reshape(a.shape), want, "fused32 N=%d c=%d" % (N, logc))


# moduli outside 34..61 bits take the generic Barrett instantiation
# (run-time word window and final shift) in every kernel, k_colq included
ANY_KIND = [(62, 16, 9), (62, 17, 10), (62, 13, 6), (33, 12, 5), (20, 11, 8), (31, 15, 8)]


@pytest.mark.parametrize("bits,log2n,logc", ANY_KIND, ids=lambda v: str(v))
def test_small_plan_other_moduli(L, small, bits, log2n, logc):
    import torch
    N, limbs, polys = 1 << log2n, 2, 2
    _install(L, log2n, logc)
    qs = L.pm_ntt_primes(N, limbs, bits)
    assert len(qs) == limbs
    fw_o, iv_o = oracle_tables(qs, N)
    prm = L.Params(N, limbs, primes=qs)
    a, b = operands(N, qs, polys, request=1800 + bits)
    x = L.to_device(a)
    L.pm_ntt_fwd(x, N, limbs, polys, qs, prm.psi_br)
    y = L.to_device(a)
    L.pm_ntt_inv(y, N, limbs, polys, qs, prm.psi_inv_br)
    da, db = L.to_device(a), L.to_device(b)
    dc, df = torch.empty_like(da), torch.empty_like(da)
    L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    L.pm_polymul_fused(da, db, df, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    _sync()
    what = "q%d N=2^%d c=%d" % (bits, log2n, logc)
    _eq(L.to_host(x).reshape(a.shape), oracle_ntt_fwd(a, qs, fw_o), "fwd " + what)
    _eq(L.to_host(y).reshape(a.shape), oracle_ntt_inv(a, qs, iv_o), "inv " + what)
    want = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    _eq(L.to_host(dc).reshape(a.shape), want, "polymul " + what)
    _eq(L.to_host(df).reshape(a.shape), want, "fused " + what)


def test_threshold_selects_plan(L, small):
    """Above the threshold the throughput plan runs; at or below it, the small plan."""
    import torch
    N, limbs = 1 << 12, 1
    qs = L.pm_ntt_primes(N, limbs)
    prm = L.Params(N, limbs, primes=qs)
    _install(L, 12, 12)
    L.pm_tune_set_small_batch(4 * N)
    a, _ = operands(N, qs, 8, request=1700)
    fw_o, _ = oracle_tables(qs, N)
    want = oracle_ntt_fwd(a, qs, fw_o)
    for polys, suffix in ((4, "s"), (8, "")):
        x = L.to_device(np.ascontiguousarray(a[:, :polys]))
        L.pm_prof_read(reset=True)
        L.pm_prof_enable(True)
        L.pm_ntt_fwd(x, N, limbs, polys, qs, prm.psi_br)
        L.pm_prof_enable(False)
        _sync()
        names = L.pm_prof_read(reset=True)
        assert list(names) == ["row_fwd_c12" + suffix], names
        _eq(L.to_host(x).reshape(1, polys, N), want[:, :polys], "threshold polys=%d" % polys)
    assert L.pm_tune_get_small(L.OP_NTT_FWD, 12) == (12, 4)
    assert L.pm_tune_get_small_batch() == 4 * N
    # a per-N limit above the global threshold: 8 polynomials now take the small plan
    L.pm_tune_set_small_limit(L.OP_NTT_FWD, 12, 8 * N)
    x = L.to_device(a)
    L.pm_prof_read(reset=True)
    L.pm_prof_enable(True)
    L.pm_ntt_fwd(x, N, limbs, 8, qs, prm.psi_br)
    L.pm_prof_enable(False)
    _sync()
    assert list(L.pm_prof_read(reset=True)) == ["row_fwd_c12s"]
    _eq(L.to_host(x).reshape(1, 8, N), want, "limit polys=8")
