"""Parity of the software-pipelined product (needs an MI355X).

pm_polymul and pm_polymul_fused (64- and 32-bit words), with rows of 2^12
words and a column radix of 2^3..2^5, split each launch group's products into
chunks and overlap the row pass of one chunk with the column passes of its
neighbours.
Every case compares each output word with the oracle, and the pipelined
result with the three-pass one (pm_tune_set_pipeline(0)) on the same inputs.
"""
import numpy as np
import pytest

from gpu_helpers import device_tables, first_mismatch, operands, oracle_polymul, oracle_tables, tuned

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    yield lib
    lib.pm_tune_set_pipeline(-1)
    for n in (15, 16, 17):
        lib.pm_tune_set(lib.OP_POLYMUL, n, 0)


def _sync():
    import torch
    torch.cuda.synchronize()


def _ws(L, N, limbs, polys):
    import torch
    nb = L.pm_polymul_workspace_bytes(N, limbs, polys)
    return torch.empty(nb // 8, dtype=torch.int64, device="cuda") if nb else None


def _assert_equal(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, "%s: %s" % (what, msg)


def _run(L, fn, a, b, N, qs, dfw, div, chunks, alias=None):
    """One call with the given pipeline setting; returns c on the host and the
    library's per-kernel launch counts."""
    import torch
    limbs, polys = a.shape[0], a.shape[1]
    da, db = L.to_device(a), L.to_device(b)
    dc = {"a": da, "b": db}.get(alias) if alias else torch.empty_like(da)
    ws = _ws(L, N, limbs, polys)
    L.pm_tune_set_pipeline(chunks)
    L.pm_prof_enable(True)
    try:
        L.pm_prof_read()                 # drop earlier launches
        fn(da, db, dc, N, limbs, polys, qs, dfw, div, ws)
        _sync()
        prof = {name: n for name, (n, _ms) in L.pm_prof_read().items()}
    finally:
        L.pm_prof_enable(False)
        L.pm_tune_set_pipeline(-1)
    return L.to_host(dc).reshape(a.shape), prof


def auto_chunks(log2n, products):
    """The built-in choice: 2 chunks from 2048 rows of 2^12 words (never at
    N = 2^17), else the three-pass form."""
    rows = products << (log2n - 12)
    return 2 if rows >= 2048 and log2n < 17 else 0


# (log2 N, limbs, polys, chunks): chunks of unequal size, chunks that end
# inside a limb, one product per chunk, more chunks asked for than products,
# more than the 64 chunks allowed, one limb, the built-in choice below and at
# its threshold
CASES = [
    (15, 3, 4, 2), (15, 5, 2, 3), (15, 3, 5, 4), (15, 4, 1, 4), (15, 2, 3, 9), (15, 2, 40, 100),
    (16, 3, 2, 2), (16, 2, 32, -1), (16, 1, 128, -1), (16, 1, 7, 3), (16, 5, 1, 5),
    (17, 3, 1, 2), (17, 2, 2, 2), (17, 1, 3, 2),
]


@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
@pytest.mark.parametrize("log2n,limbs,polys,chunks", CASES)
def test_pipelined_matches_oracle(L, log2n, limbs, polys, chunks, fused):
    N = 1 << log2n
    L.pm_tune_set(L.OP_POLYMUL, log2n, 12)
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=700 + 10 * log2n + limbs)
    fn = L.pm_polymul_fused if fused else L.pm_polymul
    got, prof = _run(L, fn, a, b, N, qs, dfw, div, chunks)
    G = min(chunks if chunks >= 0 else auto_chunks(log2n, limbs * polys), 64, limbs * polys)
    name = "pipe_fmul_c12" if fused else "pipe_mul_c12"
    if G < 2:          # the built-in choice keeps the three-pass form here
        assert name not in prof, prof
        _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "three-pass N=%d" % N)
        return
    assert prof.get(name) == G + 2, "expected %d pipelined launches, saw %s" % (G + 2, prof)
    assert not any(k.startswith("col") for k in prof), prof
    _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "pipelined N=%d" % N)
    plain, prof0 = _run(L, fn, a, b, N, qs, dfw, div, 0)
    assert name not in prof0, prof0
    _assert_equal(got, plain, "pipelined vs three-pass N=%d" % N)


@pytest.mark.parametrize("alias", ["a", "b"])
@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
def test_pipelined_aliasing(L, alias, fused):
    N, limbs, polys = 1 << 16, 3, 2
    L.pm_tune_set(L.OP_POLYMUL, 16, 12)
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=760)
    fn = L.pm_polymul_fused if fused else L.pm_polymul
    got, prof = _run(L, fn, a, b, N, qs, dfw, div, 2, alias=alias)
    assert any(k.startswith("pipe_") for k in prof), prof
    _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "c==%s" % alias)


@pytest.mark.parametrize("log2n", [16, 17])
@pytest.mark.parametrize("bits", [62, 61, 34, 33])
def test_pipelined_other_moduli(L, bits, log2n):
    """Moduli outside the 60-bit window take the general reduction kernels
    (at N = 2^17 also in the column pass shared by two lanes)."""
    N, limbs, polys = 1 << log2n, 2, 2
    L.pm_tune_set(L.OP_POLYMUL, log2n, 12)
    qs = L.pm_ntt_primes(N, limbs, bits)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=770 + bits + log2n)
    for fn in (L.pm_polymul, L.pm_polymul_fused):
        got, prof = _run(L, fn, a, b, N, qs, dfw, div, 2)
        assert any(k.startswith("pipe_") for k in prof), prof
        _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "%d-bit %s" % (bits, fn.__name__))


@pytest.mark.parametrize("log2n", [16, 17])
def test_pipelined_edge_values(L, log2n):
    """Every coefficient q - 1 (the largest products), and zeros."""
    N, limbs, polys = 1 << log2n, 2, 2
    L.pm_tune_set(L.OP_POLYMUL, log2n, 12)
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a = np.empty((limbs, polys, N), np.uint64)
    for l, q in enumerate(qs):
        a[l] = np.uint64(q - 1)
    b = a.copy()
    b[:, 1] = 0
    got, _ = _run(L, L.pm_polymul, a, b, N, qs, dfw, div, 2)
    _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "q-1 / zeros")


def test_pipelined_launch_groups(L):
    """More limbs than one launch group holds (groups of 64): each group is
    pipelined on its own."""
    N, limbs, polys = 1 << 15, 66, 1
    L.pm_tune_set(L.OP_POLYMUL, 15, 12)
    qs = L.pm_ntt_primes(N, limbs)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=790)
    got, prof = _run(L, L.pm_polymul, a, b, N, qs, dfw, div, 2)
    assert prof.get("pipe_mul_c12") == 2 * (2 + 2), prof
    plain, _ = _run(L, L.pm_polymul, a, b, N, qs, dfw, div, 0)
    _assert_equal(got, plain, "66 limbs pipelined vs three-pass")
    sample = [0, 31, 32, 63, 64, 65]
    fw_o, iv_o = oracle_tables([qs[l] for l in sample], N)
    want = oracle_polymul(a[sample], b[sample], [qs[l] for l in sample], N, fw_o, iv_o)
    _assert_equal(got[sample], want, "66 limbs, sampled limbs vs oracle")


def test_pipelined_benchmark_plan(L):
    """The tuned plans pipeline the benchmark's 2^16 product by default (here
    2 limbs x 96 pairs: 3072 rows, at the tuned threshold) and keep the
    three passes just below it (2 x 95 pairs)."""
    N, limbs, polys = 1 << 16, 2, 96
    qs = L.pm_ntt_primes(N, limbs)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=795)
    with tuned(L):
        assert L.pm_tune_get(L.OP_POLYMUL, 16) == 12
        assert L.pm_tune_get_pipeline_rows(4) == limbs * polys * 16
        got, prof = _run(L, L.pm_polymul, a, b, N, qs, dfw, div, -1)
        below, prof_b = _run(L, L.pm_polymul, a[:, :95].copy(), b[:, :95].copy(), N, qs, dfw, div, -1)
    assert prof.get("pipe_mul_c12") == 4, prof
    assert "pipe_mul_c12" not in prof_b, prof_b
    _assert_equal(below, got[:, :95], "three passes below the threshold vs pipelined")
    fw_o, iv_o = oracle_tables(qs, N)
    want = oracle_polymul(a[:, :3], b[:, :3], qs, N, fw_o, iv_o)
    _assert_equal(got[:, :3], want, "tuned plan, first three pairs per limb")


# ------------------------------------------------------------ 32-bit words --

def _run32(L, fn, a, b, N, qs, dfw, div, chunks, alias=None):
    import torch
    limbs, polys = a.shape[0], a.shape[1]
    da, db = L.to_device32(a), L.to_device32(b)
    dc = {"a": da, "b": db}.get(alias) if alias else torch.empty_like(da)
    nb = L.pm_polymul_u32_workspace_bytes(N, limbs, polys)
    ws = torch.empty(nb // 4, dtype=torch.int32, device="cuda") if nb else None
    L.pm_tune_set_pipeline(chunks)
    L.pm_prof_enable(True)
    try:
        L.pm_prof_read()
        fn(da, db, dc, N, limbs, polys, qs, dfw, div, ws)
        _sync()
        prof = {name: n for name, (n, _ms) in L.pm_prof_read().items()}
    finally:
        L.pm_prof_enable(False)
        L.pm_tune_set_pipeline(-1)
    return L.to_host32(dc).reshape(a.shape).astype(np.uint64), prof


def _moduli32(L, N, bits_list):
    qs = []
    for bits in bits_list:
        for q in L.pm_ntt_primes(N, 8, bits):
            if q not in qs:
                qs.append(q)
                break
    return qs


# (log2 N, moduli bit lengths, polys, chunks)
CASES32 = [
    (15, [30, 30, 30], 3, 2), (16, [30, 29, 28], 2, 3), (16, [30] * 2, 64, -1), (17, [29, 30], 1, 2),
]


@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
@pytest.mark.parametrize("log2n,bits,polys,chunks", CASES32)
def test_pipelined_u32(L, log2n, bits, polys, chunks, fused):
    N = 1 << log2n
    L.pm_tune_set(L.OP_POLYMUL, log2n, 12)
    qs = _moduli32(L, N, bits)
    limbs = len(qs)
    fw_o, iv_o = oracle_tables(qs, N)
    fw = np.empty((limbs, N), np.uint32)
    iv = np.empty((limbs, N), np.uint32)
    for l, q in enumerate(qs):
        fw[l], iv[l] = L.pm_make_tables_u32(q, N)
    dfw, div = L.to_device32(fw), L.to_device32(iv)
    a, b = operands(N, qs, polys, request=800 + log2n + polys)
    fn = L.pm_polymul_fused_u32 if fused else L.pm_polymul_u32
    got, prof = _run32(L, fn, a, b, N, qs, dfw, div, chunks)
    G = min(chunks if chunks >= 0 else auto_chunks(log2n, limbs * polys), 64, limbs * polys)
    name = "pipe32_fmul_c12" if fused else "pipe32_mul_c12"
    assert prof.get(name) == G + 2, "expected %d pipelined launches, saw %s" % (G + 2, prof)
    _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "pipelined u32 N=%d" % N)
    plain, prof0 = _run32(L, fn, a, b, N, qs, dfw, div, 0)
    assert name not in prof0, prof0
    _assert_equal(got, plain, "pipelined vs three-pass u32 N=%d" % N)
    if not fused:
        got_a, _ = _run32(L, fn, a, b, N, qs, dfw, div, chunks, alias="a")
        _assert_equal(got_a, plain, "pipelined u32, c==a")


def test_pipelined_u32_launch_groups(L):
    """130 limbs of 32-bit words: launch groups of 128 and 2 limbs, each
    pipelined on its own."""
    N, limbs, polys = 1 << 15, 130, 1
    L.pm_tune_set(L.OP_POLYMUL, 15, 12)
    qs = L.pm_ntt_primes(N, limbs, 30)
    assert len(qs) == limbs
    fw = np.empty((limbs, N), np.uint32)
    iv = np.empty((limbs, N), np.uint32)
    for l, q in enumerate(qs):
        fw[l], iv[l] = L.pm_make_tables_u32(q, N)
    dfw, div = L.to_device32(fw), L.to_device32(iv)
    a, b = operands(N, qs, polys, request=830)
    got, prof = _run32(L, L.pm_polymul_u32, a, b, N, qs, dfw, div, 2)
    assert prof.get("pipe32_mul_c12") == 2 * (2 + 2), prof
    plain, _ = _run32(L, L.pm_polymul_u32, a, b, N, qs, dfw, div, 0)
    _assert_equal(got, plain, "130 limbs pipelined vs three-pass")
    sample = [0, 63, 64, 127, 128, 129]
    fw_o, iv_o = oracle_tables([qs[l] for l in sample], N)
    want = oracle_polymul(a[sample], b[sample], [qs[l] for l in sample], N, fw_o, iv_o)
    _assert_equal(got[sample], want, "130 limbs, sampled limbs vs oracle")


@pytest.mark.parametrize("inplace", [False, True], ids=["c", "c==a==b"])
@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
@pytest.mark.parametrize("log2n", [15, 16, 17])
def test_pipelined_squaring(L, log2n, fused, inplace):
    """a = b: one forward column operand, the squaring rows (or the fused rows
    reading c for both), no workspace."""
    import torch
    N, limbs, polys = 1 << log2n, 3, 2
    L.pm_tune_set(L.OP_POLYMUL, log2n, 12)
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, _ = operands(N, qs, polys, request=850 + log2n)
    fn = L.pm_polymul_fused if fused else L.pm_polymul
    want = oracle_polymul(a, a, qs, N, fw_o, iv_o)
    outs = []
    for chunks in (2, 0):
        da = L.to_device(a)
        dc = da if inplace else torch.empty_like(da)
        L.pm_tune_set_pipeline(chunks)
        L.pm_prof_enable(True)
        try:
            L.pm_prof_read()
            fn(da, da, dc, N, limbs, polys, qs, dfw, div, None)
            _sync()
            prof = {k: n for k, (n, _ms) in L.pm_prof_read().items()}
        finally:
            L.pm_prof_enable(False)
            L.pm_tune_set_pipeline(-1)
        name = "pipe_fmul_c12" if fused else "pipe_sqr_c12"
        assert (prof.get(name) == 4) == (chunks == 2), prof
        outs.append(L.to_host(dc).reshape(a.shape))
    _assert_equal(outs[0], want, "pipelined squaring N=%d" % N)
    _assert_equal(outs[0], outs[1], "pipelined vs three-pass squaring N=%d" % N)
