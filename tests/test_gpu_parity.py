"""Bit-exact parity of the HIP library with the CPU oracle (needs an MI355X).

Every test calls the library through its C ABI (the ctypes binding) on
seeded synthetic operands and compares each output word with the oracle,
whose own correctness is pinned by the CPU tests. Tolerance is zero: the
arithmetic is exact, so any differing word is a failure.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import (device_tables, first_mismatch, operands, oracle_ntt_fwd, oracle_ntt_inv,
                         oracle_polymul, oracle_tables, tuned)

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


def _assert_equal(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, "%s: %s" % (what, msg)


# ------------------------------------------------------------ Barrett --

MULMOD_MODULI = [
    0x0FFFFFFFFFFFC001,          # 60-bit NTT prime (m = 60)
    (1 << 61) - 1,               # m = 61, top of the fast path
    (1 << 62) - 57,              # m = 62, needs the extra shift
    (1 << 34) - 41,              # m = 34
    (1 << 33) + 17,              # m = 34 (just above 2^33)
    (1 << 33) - 9,               # m = 33, low word window
    (1 << 30) - 35,              # m = 30
    994705409,                   # the paper's worked-example modulus
    12289, 7681, 257, 3, 2,
]


@pytest.mark.parametrize("q", MULMOD_MODULI, ids=lambda q: "q%d" % q.bit_length())
def test_barrett_mulmod(L, q):
    from paper_2209_01290_amd import synth
    n = 1 << 18
    a = synth.uniform_mod(synth.key(11, q, 0), n, q)
    b = synth.uniform_mod(synth.key(11, q, 1), n, q)
    edge = [0, 1, q - 1, max(q - 2, 0), q // 2]
    ea = np.array([x for x in edge for _ in edge], np.uint64)
    eb = np.array([y for _ in edge for y in edge], np.uint64)
    a[:ea.size], b[:eb.size] = ea, eb
    da, db = L.to_device(a), L.to_device(b)
    dc = da.clone()
    L.pm_barrett_mulmod(da, db, dc, q)
    _sync()
    _assert_equal(L.to_host(dc), oracle.default().mulmod_vec(a, b, q), "mulmod q=%d" % q)


@pytest.mark.parametrize("alias", ["c=a", "c=b", "a=b=c"])
def test_barrett_mulmod_aliased(L, alias):
    """c may alias a or b (pm.h): the in-place products equal the oracle's."""
    from paper_2209_01290_amd import synth
    q = (1 << 60) - (1 << 14) + 1
    n = (1 << 16) + 77
    a = synth.uniform_mod(synth.key(12, 0), n, q)
    b = synth.uniform_mod(synth.key(12, 1), n, q)
    da, db = L.to_device(a), L.to_device(b)
    if alias == "c=a":
        L.pm_barrett_mulmod(da, db, da, q)
        got, want = da, oracle.default().mulmod_vec(a, b, q)
    elif alias == "c=b":
        L.pm_barrett_mulmod(da, db, db, q)
        got, want = db, oracle.default().mulmod_vec(a, b, q)
    else:
        L.pm_barrett_mulmod(da, da, da, q)
        got, want = da, oracle.default().mulmod_vec(a, a, q)
    _sync()
    _assert_equal(L.to_host(got), want, "mulmod %s" % alias)


def test_barrett_worked_example(L):
    a, b, q = 994674970, 994705408, 994705409
    da, db = L.to_device(np.array([a], np.uint64)), L.to_device(np.array([b], np.uint64))
    dc = da.clone()
    L.pm_barrett_mulmod(da, db, dc, q)
    _sync()
    assert int(L.to_host(dc)[0]) == a * b % q == 30439


# ----------------------------------------------------------- transforms --

def _limbs_for(N):
    return 2 if N >= 2**15 else 3


@pytest.mark.parametrize("log2n", ALL_LOG2N)
def test_ntt_fwd_inv(L, log2n):
    N = 1 << log2n
    limbs, polys = _limbs_for(N), 2
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    fw, iv, dfw, div = device_tables(qs, N)
    assert np.array_equal(fw, fw_o) and np.array_equal(iv, iv_o), "library tables differ from oracle's"
    a, _ = operands(N, qs, polys, request=log2n)
    x = L.to_device(a)
    L.pm_ntt_fwd(x, N, limbs, polys, qs, dfw)
    _sync()
    _assert_equal(L.to_host(x).reshape(a.shape), oracle_ntt_fwd(a, qs, fw_o), "ntt_fwd N=%d" % N)
    L.pm_ntt_inv(x, N, limbs, polys, qs, div)
    _sync()
    _assert_equal(L.to_host(x).reshape(a.shape), a, "ntt_inv(ntt_fwd) N=%d" % N)
    # inverse alone, on arbitrary NTT-domain input
    y = L.to_device(a)
    L.pm_ntt_inv(y, N, limbs, polys, qs, div)
    _sync()
    _assert_equal(L.to_host(y).reshape(a.shape), oracle_ntt_inv(a, qs, iv_o), "ntt_inv N=%d" % N)


@pytest.mark.parametrize("fused", [False, True], ids=["eq2", "fused"])
@pytest.mark.parametrize("log2n", ALL_LOG2N)
def test_polymul(L, log2n, fused):
    N = 1 << log2n
    limbs, polys = _limbs_for(N), 3
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=100 + log2n)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    ws = workspace(L, N, limbs, polys)
    fn = L.pm_polymul_fused if fused else L.pm_polymul
    fn(da, db, dc, N, limbs, polys, qs, dfw, div, ws)
    _sync()
    got = L.to_host(dc).reshape(a.shape)
    want = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    _assert_equal(got, want, "polymul%s N=%d" % (" fused" if fused else "", N))
    if N <= 1024:
        o = oracle.default()
        for l in range(limbs):
            assert np.array_equal(got[l, 0], o.polymul_schoolbook(a[l, 0], b[l, 0], qs[l]))


def torch_empty_like(t):
    import torch
    return torch.empty_like(t)


def workspace(L, N, limbs, polys, stagewise=False):
    import torch
    nbytes = (L.pm_polymul_stagewise_workspace_bytes if stagewise else L.pm_polymul_workspace_bytes)(
        N, limbs, polys)
    if nbytes == 0:
        return None
    return torch.empty(nbytes // 8, dtype=torch.int64, device="cuda")


@pytest.mark.parametrize("log2n", [13, 14, 15, 16, 17])
def test_every_pass_plan(L, log2n):
    """All valid row/column splits give the same (oracle) result."""
    N = 1 << log2n
    limbs, polys = 2, 2
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=200 + log2n)
    want_mul = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    want_fwd = oracle_ntt_fwd(a, qs, fw_o)
    da, db = L.to_device(a), L.to_device(b)
    try:
        for logc in range(8, min(log2n, 14) + 1):
            if log2n - logc > 5:
                continue
            for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
                L.pm_tune_set(op, log2n, logc)
            dc = torch_empty_like(da)
            L.pm_polymul(da, db, dc, N, limbs, polys, qs, dfw, div, workspace(L, N, limbs, polys))
            df = torch_empty_like(da)
            L.pm_polymul_fused(da, db, df, N, limbs, polys, qs, dfw, div, workspace(L, N, limbs, polys))
            x = da.clone()
            L.pm_ntt_fwd(x, N, limbs, polys, qs, dfw)
            _sync()
            _assert_equal(L.to_host(dc).reshape(a.shape), want_mul, "polymul N=%d logc=%d" % (N, logc))
            _assert_equal(L.to_host(df).reshape(a.shape), want_mul, "fused N=%d logc=%d" % (N, logc))
            _assert_equal(L.to_host(x).reshape(a.shape), want_fwd, "ntt_fwd N=%d logc=%d" % (N, logc))
            L.pm_ntt_inv(x, N, limbs, polys, qs, div)
            _sync()
            _assert_equal(L.to_host(x).reshape(a.shape), a, "roundtrip N=%d logc=%d" % (N, logc))
    finally:
        for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
            L.pm_tune_set(op, log2n, 0)


@pytest.mark.parametrize("log2n", [1, 4, 10, 14, 16])
def test_stagewise(L, log2n):
    N = 1 << log2n
    limbs, polys = 2, 2
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=300 + log2n)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul_stagewise(da, db, dc, N, limbs, polys, qs, dfw, div, workspace(L, N, limbs, polys, True))
    _sync()
    _assert_equal(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o),
                  "stagewise N=%d" % N)


@pytest.mark.parametrize("log2n", [10, 16])
@pytest.mark.parametrize("path", ["eq2", "stagewise", "alg8"])
def test_aliasing(L, log2n, path):
    N = 1 << log2n
    limbs, polys = 2, 2
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=400 + log2n)
    fn = {"eq2": L.pm_polymul, "stagewise": L.pm_polymul_stagewise, "alg8": L.pm_polymul_fused}[path]
    ws = workspace(L, N, limbs, polys, path == "stagewise")
    want_ab = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    want_aa = oracle_polymul(a, a, qs, N, fw_o, iv_o)
    # c aliases a
    da, db = L.to_device(a), L.to_device(b)
    fn(da, db, da, N, limbs, polys, qs, dfw, div, ws)
    _sync()
    _assert_equal(L.to_host(da).reshape(a.shape), want_ab, "c==a")
    # c aliases b
    da, db = L.to_device(a), L.to_device(b)
    fn(da, db, db, N, limbs, polys, qs, dfw, div, ws)
    _sync()
    _assert_equal(L.to_host(db).reshape(a.shape), want_ab, "c==b")
    # squaring in place
    da = L.to_device(a)
    fn(da, da, da, N, limbs, polys, qs, dfw, div, None)
    _sync()
    _assert_equal(L.to_host(da).reshape(a.shape), want_aa, "c==a==b")


def test_many_limbs_chunked(L):
    """More limbs than fit one launch's kernel arguments (chunks of 64)."""
    N, limbs, polys = 256, 70, 1
    qs = L.pm_ntt_primes(N, limbs)
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, request=500)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul(da, db, dc, N, limbs, polys, qs, dfw, div, None)
    x = da.clone()
    L.pm_ntt_fwd(x, N, limbs, polys, qs, dfw)
    _sync()
    _assert_equal(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "70 limbs")
    _assert_equal(L.to_host(x).reshape(a.shape), oracle_ntt_fwd(a, qs, fw_o), "70 limbs fwd")


ODD_MODULI = [  # (bits of the prime search, log2 N)
    (62, 16), (62, 10), (61, 16), (35, 14), (34, 12), (33, 12), (31, 16), (30, 10), (20, 8),
]


@pytest.mark.parametrize("bits,log2n", ODD_MODULI, ids=lambda v: str(v))
def test_moduli_of_other_lengths(L, bits, log2n):
    N = 1 << log2n
    qs = L.pm_ntt_primes(N, 2, bits)
    assert len(qs) == 2
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, 2, request=600 + bits)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul(da, db, dc, N, 2, 2, qs, dfw, div, workspace(L, N, 2, 2))
    x = da.clone()
    L.pm_ntt_fwd(x, N, 2, 2, qs, dfw)
    _sync()
    _assert_equal(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "polymul")
    _assert_equal(L.to_host(x).reshape(a.shape), oracle_ntt_fwd(a, qs, fw_o), "ntt_fwd")


@pytest.mark.parametrize("small_q,log2n", [(12289, 11), (7681, 8), (257, 7), (65537, 15), (97, 4)])
def test_small_primes(L, small_q, log2n):
    N = 1 << log2n
    qs = [small_q]
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, 3, request=700 + log2n)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul(da, db, dc, N, 1, 3, qs, dfw, div, workspace(L, N, 1, 3))
    _sync()
    _assert_equal(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "q=%d" % small_q)


@pytest.mark.parametrize("log2n", [10, 16, 17])
def test_edge_values(L, log2n):
    """All-(q-1) operands, zeros, and x^(N-1) * x = -1."""
    N = 1 << log2n
    qs = L.pm_ntt_primes(N, 1)
    q = qs[0]
    fw_o, iv_o = oracle_tables(qs, N)
    _, _, dfw, div = device_tables(qs, N)
    a = np.full((1, 3, N), q - 1, np.uint64)
    b = np.full((1, 3, N), q - 1, np.uint64)
    b[0, 1] = 0
    a[0, 2] = 0
    b[0, 2] = 0
    a[0, 2, N - 1] = 1
    b[0, 2, 1 % N] = 1
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul(da, db, dc, N, 1, 3, qs, dfw, div, workspace(L, N, 1, 3))
    _sync()
    got = L.to_host(dc).reshape(a.shape)
    _assert_equal(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "edge N=%d" % N)
    assert np.all(got[0, 1] == 0)
    mono = np.zeros(N, np.uint64)
    mono[0] = q - 1 if N > 1 else 0
    assert np.array_equal(got[0, 2], mono)


# ------------------------------------------------- workload-size parity --

def test_config1_single_polymul(L):
    """N=1024, one 60-bit prime, one pair, against the schoolbook product."""
    N = 1024
    qs = L.pm_ntt_primes(N, 1)
    assert qs[0] == 2**60 - 2**14 + 1
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, 1, seed=220901290 + 1)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul(da, db, dc, N, 1, 1, qs, dfw, div, None)
    _sync()
    want = oracle.default().polymul_schoolbook(a[0, 0], b[0, 0], qs[0])
    _assert_equal(L.to_host(dc).reshape(N), want, "config 1")


def test_config2_stagewise_full_size(L):
    """N=2^14, 32 limbs, plain per-stage path at full size; oracle on sampled limbs."""
    N, limbs, polys = 2**14, 32, 1
    qs = L.pm_ntt_primes(N, limbs)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, seed=220901290 + 2)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    L.pm_polymul_stagewise(da, db, dc, N, limbs, polys, qs, dfw, div, workspace(L, N, limbs, polys, True))
    dc2 = torch_empty_like(da)
    L.pm_polymul(da, db, dc2, N, limbs, polys, qs, dfw, div, workspace(L, N, limbs, polys))
    _sync()
    got, got2 = L.to_host(dc).reshape(a.shape), L.to_host(dc2).reshape(a.shape)
    o = oracle.default()
    for l in [0, 13, 31]:
        fw, iv = o.psi_tables(qs[l], N)
        want = o.polymul_ntt(a[l, 0], b[l, 0], qs[l], fw, iv)
        _assert_equal(got[l, 0], want, "config 2 stagewise limb %d" % l)
        _assert_equal(got2[l, 0], want, "config 2 fused limb %d" % l)
    rng = np.random.default_rng(2)
    for l in rng.integers(0, limbs, 6):
        for k in rng.integers(0, N, 4):
            assert int(got[l, 0, k]) == o.polymul_coeff(a[l, 0], b[l, 0], qs[l], int(k))


def test_config3_full_size(L):
    """N=2^16, 48 limbs x 8 pairs (the benchmark shape) plus the standalone
    forward NTT of the a operands: every one of the 384 products, in the
    software-pipelined form the benchmark times and in the three-pass form,
    and every forward transform, word for word against the oracle."""
    from gpu_helpers import oracle_parallel
    N, limbs, polys = 2**16, 48, 8
    qs = L.pm_ntt_primes(N, limbs)
    _, _, dfw, div = device_tables(qs, N)
    a, b = operands(N, qs, polys, seed=220901290 + 3)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch_empty_like(da)
    got = {}
    with tuned(L):                       # the plans the benchmark runs
        for form, chunks in (("pipelined", -1), ("three-pass", 0)):
            L.pm_tune_set_pipeline(chunks)
            dc.zero_()
            L.pm_polymul(da, db, dc, N, limbs, polys, qs, dfw, div, workspace(L, N, limbs, polys))
            _sync()
            got[form] = L.to_host(dc).reshape(a.shape)
        x = da.clone()
        L.pm_ntt_fwd(x, N, limbs, polys, qs, dfw)
        _sync()
    fwd = L.to_host(x).reshape(a.shape)
    o = oracle.default()
    tables = oracle_parallel(lambda q: o.psi_tables(q, N), qs)

    def check(lp):
        l, p = lp
        fw, iv = tables[l]
        want = o.polymul_ntt(a[l, p], b[l, p], qs[l], fw, iv)
        bad = [form for form in got if not np.array_equal(got[form][l, p], want)]
        if not np.array_equal(fwd[l, p], o.ntt_fwd(a[l, p], qs[l], fw)):
            bad.append("ntt_fwd")
        return bad

    pairs = [(l, p) for l in range(limbs) for p in range(polys)]
    res = oracle_parallel(check, pairs)
    wrong = [(lp, bad) for lp, bad in zip(pairs, res) if bad]
    assert not wrong, "%d of 384 products differ from the oracle, first: %s" % (len(wrong), wrong[0])