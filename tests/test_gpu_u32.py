"""Bit-exact parity of the 32-bit word path (moduli up to 30 bits, the word
size of the paper's 30-bit experiments; Alg. 4 with beta = 32) with the CPU
oracle, through the C ABI. Operands are drawn below q by the shared seeded
generator and handed to the oracle as 64-bit words; the oracle's result must
equal the device's word for word (tolerance zero)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import first_mismatch, operands, oracle_ntt_fwd, oracle_ntt_inv, oracle_polymul, oracle_tables, tuned

pytestmark = pytest.mark.gpu

ALL_LOG2N = list(range(1, 18))


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


def _sync():
    import torch
    torch.cuda.synchronize()


def _eq(got, want, what):
    msg = first_mismatch(np.asarray(got, dtype=np.uint64), np.asarray(want, dtype=np.uint64))
    assert msg is None, "%s: %s" % (what, msg)


def _tables32(L, qs, N):
    fw = np.empty((len(qs), N), np.uint32)
    iv = np.empty((len(qs), N), np.uint32)
    for l, q in enumerate(qs):
        fw[l], iv[l] = L.pm_make_tables_u32(q, N)
    return L.to_device32(fw), L.to_device32(iv)


def _ws(L, N, limbs, polys):
    import torch
    n = L.pm_polymul_u32_workspace_bytes(N, limbs, polys)
    return torch.empty(n // 4, dtype=torch.int32, device="cuda") if n else None


def _moduli(L, N, bits_list):
    qs = []
    for bits in bits_list:
        for q in L.pm_ntt_primes(N, 4, bits):
            if q not in qs:
                qs.append(q)
                break
    assert len(qs) == len(bits_list)
    return qs


# 30-bit moduli take the extra final shift (KIND_ANY); 28/29-bit ones do not.
BITS = {"q30": [30, 30], "q29_28": [29, 28], "mixed": [30, 27]}


@pytest.mark.parametrize("bits", list(BITS), ids=list(BITS))
@pytest.mark.parametrize("log2n", ALL_LOG2N)
def test_ntt_u32(L, log2n, bits):
    N = 1 << log2n
    qs = _moduli(L, N, BITS[bits])
    limbs, polys = len(qs), 2
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a, _ = operands(N, qs, polys, request=500 + log2n)
    x = L.to_device32(a)
    L.pm_ntt_fwd_u32(x, N, limbs, polys, qs, dfw)
    _sync()
    _eq(L.to_host32(x).reshape(a.shape), oracle_ntt_fwd(a, qs, fw_o), "ntt_fwd_u32 N=%d" % N)
    L.pm_ntt_inv_u32(x, N, limbs, polys, qs, div)
    _sync()
    _eq(L.to_host32(x).reshape(a.shape), a, "roundtrip u32 N=%d" % N)
    y = L.to_device32(a)
    L.pm_ntt_inv_u32(y, N, limbs, polys, qs, div)
    _sync()
    _eq(L.to_host32(y).reshape(a.shape), oracle_ntt_inv(a, qs, iv_o), "ntt_inv_u32 N=%d" % N)


@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
@pytest.mark.parametrize("bits", list(BITS), ids=list(BITS))
@pytest.mark.parametrize("log2n", ALL_LOG2N)
def test_polymul_u32(L, log2n, bits, fused):
    import torch
    N = 1 << log2n
    qs = _moduli(L, N, BITS[bits])
    limbs, polys = len(qs), 3
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a, b = operands(N, qs, polys, request=600 + log2n)
    da, db = L.to_device32(a), L.to_device32(b)
    dc = torch.empty_like(da)
    fn = L.pm_polymul_fused_u32 if fused else L.pm_polymul_u32
    fn(da, db, dc, N, limbs, polys, qs, dfw, div, _ws(L, N, limbs, polys))
    _sync()
    got = L.to_host32(dc).reshape(a.shape)
    _eq(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "polymul%s_u32 N=%d" % ("_fused" if fused else "", N))
    if N <= 512:
        o = oracle.default()
        assert np.array_equal(got[0, 0].astype(np.uint64), o.polymul_schoolbook(a[0, 0], b[0, 0], qs[0]))


@pytest.mark.parametrize("log2n", [13, 14, 15, 16, 17])
def test_every_pass_plan_u32(L, log2n):
    import torch
    N = 1 << log2n
    qs = _moduli(L, N, [30, 29])
    limbs, polys = 2, 2
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a, b = operands(N, qs, polys, request=700 + log2n)
    want = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    want_fwd = oracle_ntt_fwd(a, qs, fw_o)
    da, db = L.to_device32(a), L.to_device32(b)
    try:
        for logc in range(8, min(log2n, 14) + 1):
            if log2n - logc > 5:
                continue
            for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
                L.pm_tune_set(op, log2n, logc)
            dc = torch.empty_like(da)
            L.pm_polymul_u32(da, db, dc, N, limbs, polys, qs, dfw, div, _ws(L, N, limbs, polys))
            df = torch.empty_like(da)
            L.pm_polymul_fused_u32(da, db, df, N, limbs, polys, qs, dfw, div, _ws(L, N, limbs, polys))
            x = da.clone()
            L.pm_ntt_fwd_u32(x, N, limbs, polys, qs, dfw)
            _sync()
            _eq(L.to_host32(dc).reshape(a.shape), want, "polymul_u32 N=%d logc=%d" % (N, logc))
            _eq(L.to_host32(df).reshape(a.shape), want, "fused_u32 N=%d logc=%d" % (N, logc))
            _eq(L.to_host32(x).reshape(a.shape), want_fwd, "ntt_fwd_u32 N=%d logc=%d" % (N, logc))
            L.pm_ntt_inv_u32(x, N, limbs, polys, qs, div)
            _sync()
            _eq(L.to_host32(x).reshape(a.shape), a, "roundtrip u32 N=%d logc=%d" % (N, logc))
    finally:
        for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
            L.pm_tune_set(op, log2n, 0)


@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
@pytest.mark.parametrize("log2n", [10, 16])
@pytest.mark.parametrize("alias", ["c=a", "c=b", "a=b", "a=b=c"])
def test_aliasing_u32(L, log2n, alias, fused):
    N = 1 << log2n
    qs = _moduli(L, N, [30, 28])
    limbs, polys = 2, 2
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a, b = operands(N, qs, polys, request=800 + log2n)
    if alias.startswith("a=b"):
        b = a
    da, db = L.to_device32(a), L.to_device32(b)
    if alias == "c=a":
        dc = da
    elif alias == "c=b":
        dc = db
    elif alias == "a=b":
        db = da
        dc = L.to_device32(np.zeros_like(a))
    else:
        db = dc = da
    fn = L.pm_polymul_fused_u32 if fused else L.pm_polymul_u32
    fn(da, db, dc, N, limbs, polys, qs, dfw, div, _ws(L, N, limbs, polys))
    _sync()
    _eq(L.to_host32(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "u32 %s N=%d" % (alias, N))


def test_many_limbs_chunked_u32(L):
    """More limbs than one launch group holds (128 moduli for 32-bit words)."""
    import torch
    N, limbs, polys = 1024, 130, 1
    qs = L.pm_ntt_primes(N, limbs, 30)
    assert len(qs) == limbs
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a, b = operands(N, qs, polys, request=900)
    da, db = L.to_device32(a), L.to_device32(b)
    dc = torch.empty_like(da)
    L.pm_polymul_u32(da, db, dc, N, limbs, polys, qs, dfw, div, _ws(L, N, limbs, polys))
    _sync()
    _eq(L.to_host32(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "130 limbs u32")


@pytest.mark.parametrize("small_q,log2n", [(12289, 11), (7681, 8), (257, 7), (65537, 15), (97, 4), (17, 3)])
def test_small_moduli_u32(L, small_q, log2n):
    import torch
    N = 1 << log2n
    qs = [small_q]
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a, b = operands(N, qs, 2, request=1000 + small_q)
    da, db = L.to_device32(a), L.to_device32(b)
    dc = torch.empty_like(da)
    L.pm_polymul_u32(da, db, dc, N, 1, 2, qs, dfw, div, _ws(L, N, 1, 2))
    _sync()
    _eq(L.to_host32(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "u32 q=%d" % small_q)


@pytest.mark.parametrize("log2n", [10, 16, 17])
def test_edge_values_u32(L, log2n):
    """All-zero, all-(q-1) and single-monomial operands at the largest 30-bit prime."""
    import torch
    N = 1 << log2n
    qs = _moduli(L, N, [30])
    q = qs[0]
    fw_o, iv_o = oracle_tables(qs, N)
    dfw, div = _tables32(L, qs, N)
    a = np.zeros((1, 4, N), np.uint64)
    b = np.zeros((1, 4, N), np.uint64)
    a[0, 1] = q - 1
    b[0, 1] = q - 1
    a[0, 2] = q - 1
    b[0, 2, N - 1] = q - 1              # (q-1) * x^(N-1) wraps negacyclically
    a[0, 3, 0] = 1
    b[0, 3] = np.arange(N, dtype=np.uint64) % q
    da, db = L.to_device32(a), L.to_device32(b)
    dc = torch.empty_like(da)
    L.pm_polymul_u32(da, db, dc, N, 1, 4, qs, dfw, div, _ws(L, N, 1, 4))
    _sync()
    got = L.to_host32(dc).reshape(a.shape)
    _eq(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "u32 edges N=%d" % N)
    assert not got[0, 0].any()
    assert np.array_equal(got[0, 3], b[0, 3])


def test_words32_full_size(L):
    """The 32-bit benchmark shape: N = 2^16, 96 limbs of 30-bit primes x 8 pairs
    (two launches of 64 + 32 limbs), with the packaged pass plans installed;
    oracle on sampled polynomials (a limb of each launch) and coefficients."""
    import torch
    N, limbs, polys = 1 << 16, 96, 8
    with tuned(L):
        prm = L.Params32(N, limbs, bits=30)
        qs = prm.q
        a, b = operands(N, qs, polys, request=2000)
        da, db = L.to_device32(a), L.to_device32(b)
        dc = torch.empty_like(da)
        L.pm_polymul_u32(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
        _sync()
        got = L.to_host32(dc).reshape(a.shape)
        o = oracle.default()
        for l, p in [(0, 0), (63, 5), (64, 2), (95, 7)]:
            fw, iv = o.psi_tables(qs[l], N)
            _eq(got[l, p], o.polymul_ntt(a[l, p], b[l, p], qs[l], fw, iv), "words32 (%d,%d)" % (l, p))
        rng = np.random.default_rng(32)
        for _ in range(8):
            l, p, k = int(rng.integers(limbs)), int(rng.integers(polys)), int(rng.integers(N))
            assert int(got[l, p, k]) == o.polymul_coeff(a[l, p], b[l, p], qs[l], k), (l, p, k)
