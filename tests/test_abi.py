"""The C-ABI library on the CPU: it loads, exports every symbol the header
declares, rejects invalid arguments before touching a device, and its host
parameter helpers agree with the oracle. No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pm.h")


@pytest.fixture(scope="module")
def L():
    from paper_2209_01290_amd import lib
    if not os.path.exists(lib.LIB_PATH):
        pytest.fail("libpm.so is not built (python -m paper_2209_01290_amd.build)")
    lib.load()
    return lib


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 12
    raw = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), "libpm.so does not export " + n
    assert set(L.exported_symbols()) <= set(names)


FAKE = ctypes.c_void_p(0x10000)      # never dereferenced: validation fails first


def _rc(f, *args):
    return f(*args)


def test_invalid_arguments_rejected_on_host(L):
    lib = L.load()
    q = (ctypes.c_uint64 * 1)(0x0FFFFFFFFFFFC001)
    # N not a power of two / out of range
    for N in [0, 1, 3, 1000, 1 << 18]:
        assert lib.pm_polymul(FAKE, FAKE, FAKE, N, 1, 1, q, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
        assert lib.pm_ntt_fwd(FAKE, N, 1, 1, q, FAKE, None) == L.PM_EINVAL
        assert "N must be" in lib.pm_last_error().decode()
    # even q, q >= 2^62, 2N not dividing q-1
    for bad in [0x0FFFFFFFFFFFC000, (1 << 62) + 1, 0x0FFFFFFFFFFFC001 + 2]:
        qb = (ctypes.c_uint64 * 1)(bad)
        assert lib.pm_polymul(FAKE, FAKE, FAKE, 1024, 1, 1, qb, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
    # zero counts, null and misaligned pointers
    assert lib.pm_polymul(FAKE, FAKE, FAKE, 1024, 0, 1, q, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
    assert lib.pm_polymul(None, FAKE, FAKE, 1024, 1, 1, q, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
    assert lib.pm_polymul(ctypes.c_void_p(0x10004), FAKE, FAKE, 1024, 1, 1, q, FAKE, FAKE, FAKE,
                          None) == L.PM_EINVAL
    assert "aligned" in lib.pm_last_error().decode()
    # a 2-D split needs the workspace
    assert lib.pm_polymul(FAKE, ctypes.c_void_p(0x20000), FAKE, 1 << 16, 1, 1,
                          (ctypes.c_uint64 * 1)(0x0FFFFFFFFFFC0001), FAKE, FAKE, None, None) == L.PM_EINVAL
    assert lib.pm_barrett_mulmod(FAKE, FAKE, FAKE, 0, 97, None) == L.PM_EINVAL
    assert lib.pm_barrett_mulmod(FAKE, FAKE, FAKE, 8, 1 << 62, None) == L.PM_EINVAL
    assert lib.pm_barrett_mulmod(FAKE, FAKE, FAKE, 8, 1, None) == L.PM_EINVAL


def test_tuning_table(L):
    for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
        assert L.pm_tune_get(op, 16) == 12
        with pytest.raises(L.PMError):
            L.pm_tune_set(op, 16, 10)        # 64 rows: column radix above 2^5
        with pytest.raises(L.PMError):
            L.pm_tune_set(op, 12, 7)         # fewer than 256 columns
        L.pm_tune_set(op, 16, 13)
        assert L.pm_tune_get(op, 16) == 13
        L.pm_tune_set(op, 16, 0)
        assert L.pm_tune_get(op, 16) == 12


def test_workspace_sizes(L):
    assert L.pm_polymul_workspace_bytes(1024, 4, 2) == 0
    assert L.pm_polymul_workspace_bytes(1 << 16, 48, 8) == (1 << 16) * 48 * 8 * 8
    assert L.pm_polymul_stagewise_workspace_bytes(1 << 14, 32, 1) == (1 << 14) * 32 * 8


@pytest.mark.parametrize("N,count", [(1024, 1), (1 << 14, 32), (1 << 16, 48), (1 << 17, 60)])
def test_host_params_match_oracle(L, N, count):
    o = oracle.default()
    qs = L.pm_ntt_primes(N, count)
    assert qs == o.ntt_primes(N, count)
    for q in qs[:2]:
        assert L.pm_find_psi(q, N) == o.find_psi(q, N)
        if N <= 1 << 14:
            f, i = L.pm_make_tables(q, N)
            f2, i2 = o.psi_tables(q, N)
            assert np.array_equal(f, f2) and np.array_equal(i, i2)


def test_tune_db_applies(L, tmp_path):
    import json
    from paper_2209_01290_amd import tune
    assert tune.candidates(16) == [11, 12, 13, 14] and tune.candidates(8) == [8]
    db = {"choices": {"polymul": {"15": 11}, "ntt_fwd": {"13": 8}}}
    p = tmp_path / "db.json"
    p.write_text(json.dumps(db))
    try:
        assert L.apply_tune_db(str(p)) == 2
        assert L.pm_tune_get(L.OP_POLYMUL, 15) == 11 and L.pm_tune_get(L.OP_NTT_FWD, 13) == 8
        assert L.apply_tune_db(str(tmp_path / "missing.json")) == 0
        # the packaged database only names implemented splits
        shipped = json.load(open(tune.DEFAULT_DB))
        for name, table in shipped["choices"].items():
            for log2n, logc in table.items():
                assert logc in tune.candidates(int(log2n))
        for name, table in shipped["small"]["choices"].items():
            for log2n, plan in table.items():
                assert tuple(plan) in tune.small_candidates(int(log2n))
        n = L.apply_tune_db()
        assert n == sum(len(t) for t in shipped["choices"].values()) + \
            sum(len(t) for t in shipped["small"]["choices"].values()) + \
            sum(len(t) for t in shipped["small"].get("limits", {}).values()) + \
            len(shipped.get("pipeline", {}).get("min_rows", {}))
        for logr, rows in shipped.get("pipeline", {}).get("min_rows", {}).items():
            assert L.pm_tune_get_pipeline_rows(int(logr)) == rows
        assert L.pm_tune_get_small_batch() == shipped["small"]["max_words"] > 0
        assert L.pm_tune_get_small(L.OP_POLYMUL, 16) == tuple(shipped["small"]["choices"]["polymul"]["16"])
        ops = {"polymul": L.OP_POLYMUL, "ntt_fwd": L.OP_NTT_FWD, "ntt_inv": L.OP_NTT_INV}
        for name, table in shipped["small"].get("limits", {}).items():
            for log2n, words in table.items():
                assert L.pm_tune_get_small_limit(ops[name], int(log2n)) == words
    finally:
        for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
            for n in range(1, 18):
                L.pm_tune_set(op, n, 0)
                L.pm_tune_set_small(op, n, 0, 0)
                L.pm_tune_set_small_limit(op, n, 0)
        L.pm_tune_set_small_batch(0)
        for logr in (3, 4, 5):
            L.pm_tune_set_pipeline_rows(logr, 0)


def test_u32_invalid_arguments_rejected_on_host(L):
    lib = L.load()
    q30 = L.pm_ntt_primes(1024, 1, 30)[0]
    q = (ctypes.c_uint32 * 1)(q30)
    for N in [0, 1, 3, 1 << 18]:
        assert lib.pm_polymul_u32(FAKE, FAKE, FAKE, N, 1, 1, q, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
        assert lib.pm_ntt_fwd_u32(FAKE, N, 1, 1, q, FAKE, None) == L.PM_EINVAL
    # a 31-bit modulus (Alg. 4 on 32-bit words needs len(q) <= 30), even q, 2N not dividing q-1
    q31 = L.pm_ntt_primes(1024, 1, 31)[0]
    for bad in [q31, q30 - 1, q30 + 2]:
        qb = (ctypes.c_uint32 * 1)(bad)
        assert lib.pm_polymul_u32(FAKE, FAKE, FAKE, 1024, 1, 1, qb, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
        assert lib.pm_ntt_inv_u32(FAKE, 1024, 1, 1, qb, FAKE, None) == L.PM_EINVAL
    # 4-byte alignment suffices for 32-bit words; 2-byte does not
    assert lib.pm_polymul_u32(ctypes.c_void_p(0x10002), FAKE, FAKE, 1024, 1, 1, q, FAKE, FAKE, FAKE,
                              None) == L.PM_EINVAL
    assert "aligned" in lib.pm_last_error().decode()
    # a 2-D split needs the workspace
    q16 = (ctypes.c_uint32 * 1)(L.pm_ntt_primes(1 << 16, 1, 30)[0])
    assert lib.pm_polymul_u32(FAKE, ctypes.c_void_p(0x20000), FAKE, 1 << 16, 1, 1, q16, FAKE, FAKE, None,
                              None) == L.PM_EINVAL
    assert "workspace" in lib.pm_last_error().decode()
    assert L.pm_polymul_u32_workspace_bytes(1 << 16, 4, 2) == (1 << 16) * 4 * 2 * 4
    assert L.pm_polymul_u32_workspace_bytes(1024, 4, 2) == 0


@pytest.mark.parametrize("N,bits", [(1024, 30), (1 << 14, 29), (1 << 16, 28)])
def test_u32_tables_match_oracle(L, N, bits):
    o = oracle.default()
    q = L.pm_ntt_primes(N, 1, bits)[0]
    assert q < 1 << bits and q == o.ntt_primes(N, 1, bits)[0]
    f, i = L.pm_make_tables_u32(q, N)
    assert f.dtype == np.uint32
    if N <= 1 << 14:
        f2, i2 = o.psi_tables(q, N)
        assert np.array_equal(f.astype(np.uint64), f2) and np.array_equal(i.astype(np.uint64), i2)
    with pytest.raises(L.PMError):
        L.pm_make_tables_u32(L.pm_ntt_primes(N, 1, 31)[0], N)


def test_il_invalid_arguments_and_workspace(L):
    lib = L.load()
    q = (ctypes.c_uint64 * 1)(0x0FFFFFFFFFFFC001)
    for N in [0, 3, 1 << 18]:
        assert lib.pm_polymul_il(FAKE, FAKE, FAKE, N, 1, 1, q, FAKE, FAKE, FAKE, None) == L.PM_EINVAL
        assert lib.pm_ntt_fwd_il(FAKE, N, 1, 1, q, FAKE, None) == L.PM_EINVAL
    assert lib.pm_ntt_inv_il(FAKE, 1024, 1, 0, q, FAKE, None) == L.PM_EINVAL
    # up to 2^5 stages run as one fused block: no workspace below N = 64
    assert L.pm_polymul_il_workspace_bytes(32, 3, 7) == 0
    assert L.pm_polymul_il_workspace_bytes(64, 3, 7) == 64 * 3 * 7 * 8
    assert lib.pm_polymul_il(FAKE, ctypes.c_void_p(0x20000), FAKE, 1024, 1, 1, q, FAKE, FAKE, None,
                             None) == L.PM_EINVAL
    assert "workspace" in lib.pm_last_error().decode()


def test_small_plan_table(L):
    lib = L.load()
    try:
        assert L.pm_tune_get_small(L.OP_NTT_FWD, 14) == (0, 0)
        assert L.pm_tune_get_small_batch() == 0
        L.pm_tune_set_small(L.OP_NTT_FWD, 14, 10, 4)
        assert L.pm_tune_get_small(L.OP_NTT_FWD, 14) == (10, 4)
        L.pm_tune_set_small(L.OP_POLYMUL, 13, 13, 16)
        assert L.pm_tune_get_small(L.OP_POLYMUL, 13) == (13, 16)
        # 4 words per thread: rows of 2^5..2^12, column passes of 2^2..2^7 rows
        # (2 rows only with >= 256 columns); 16 words: the throughput splits
        for bad in [(14, 14, 4), (4, 4, 4), (17, 9, 4), (8, 7, 4), (12, 7, 16), (10, 10, 8)]:
            assert lib.pm_tune_set_small(L.OP_NTT_FWD, *bad) == L.PM_EINVAL, bad
        for good in [(16, 10, 4), (13, 6, 4), (9, 5, 4), (9, 8, 4), (17, 10, 4)]:
            assert lib.pm_tune_set_small(L.OP_NTT_INV, *good) == 0, good
            assert L.pm_tune_get_small(L.OP_NTT_INV, good[0]) == good[1:]
        # a small plan changes the workspace only for batches under the threshold
        N = 1 << 13
        L.pm_tune_set_small(L.OP_POLYMUL, 13, 9, 4)
        assert L.pm_polymul_workspace_bytes(N, 1, 1) == 0
        L.pm_tune_set_small_batch(N)
        assert L.pm_polymul_workspace_bytes(N, 1, 1) == N * 8
        assert L.pm_polymul_workspace_bytes(N, 1, 2) == 0
        # a per-(op, N) limit replaces the global threshold for that (op, N) only
        L.pm_tune_set_small_limit(L.OP_POLYMUL, 13, 4 * N)
        assert L.pm_tune_get_small_limit(L.OP_POLYMUL, 13) == 4 * N
        assert L.pm_tune_get_small_limit(L.OP_NTT_FWD, 13) == 0
        assert L.pm_polymul_workspace_bytes(N, 1, 4) == 4 * N * 8
        assert L.pm_polymul_workspace_bytes(N, 2, 2) == 4 * N * 8
        assert L.pm_polymul_workspace_bytes(N, 1, 8) == 0
        L.pm_tune_set_small_limit(L.OP_POLYMUL, 13, 0)
        assert L.pm_polymul_workspace_bytes(N, 1, 4) == 0 and L.pm_polymul_workspace_bytes(N, 1, 1) == N * 8
        for bad in [(3, 13), (-1, 13), (L.OP_POLYMUL, 0), (L.OP_POLYMUL, 18)]:
            assert lib.pm_tune_set_small_limit(bad[0], bad[1], 1) == L.PM_EINVAL, bad
            assert L.pm_tune_get_small_limit(*bad) == 0
    finally:
        for op in (L.OP_NTT_FWD, L.OP_NTT_INV, L.OP_POLYMUL):
            for n in range(1, 18):
                L.pm_tune_set_small(op, n, 0, 0)
                L.pm_tune_set_small_limit(op, n, 0)
        L.pm_tune_set_small_batch(0)


def test_pipeline_setting():
    """pm_tune_set_pipeline: -1 (any negative) = built-in choice, 0/1 = off,
    G >= 2 = G chunks; the workspace does not depend on it."""
    from paper_2209_01290_amd import lib as L
    L.load()
    try:
        assert L.pm_tune_get_pipeline() == -1
        N = 1 << 16
        ws = L.pm_polymul_workspace_bytes(N, 48, 8)
        for g, want in [(0, 0), (1, 1), (3, 3), (-7, -1), (2, 2)]:
            L.pm_tune_set_pipeline(g)
            assert L.pm_tune_get_pipeline() == want
            assert L.pm_polymul_workspace_bytes(N, 48, 8) == ws
    finally:
        L.pm_tune_set_pipeline(-1)


def test_pipeline_rows_setting():
    """pm_tune_set_pipeline_rows: per column radix 2^3..2^5, 0 restores the
    built-in threshold (2048; never for radix 32), other radices are rejected;
    the packaged database installs its tuned thresholds."""
    from paper_2209_01290_amd import lib as L
    L.load()
    before = {r: L.pm_tune_get_pipeline_rows(r) for r in (3, 4, 5)}
    try:
        for r in (3, 4, 5):
            L.pm_tune_set_pipeline_rows(r, 0)
        assert [L.pm_tune_get_pipeline_rows(r) for r in (3, 4, 5)] == [2048, 2048, (1 << 64) - 1]
        L.pm_tune_set_pipeline_rows(4, 12345)
        assert L.pm_tune_get_pipeline_rows(4) == 12345
        L.pm_tune_set_pipeline_rows(5, (1 << 64) - 1)
        assert L.pm_tune_get_pipeline_rows(5) == (1 << 64) - 1
        for bad in (0, 2, 6, 17):
            with pytest.raises(L.PMError) as ei:
                L.pm_tune_set_pipeline_rows(bad, 100)
            assert ei.value.code == L.PM_EINVAL
            assert L.pm_tune_get_pipeline_rows(bad) == 0
        import json, os
        db = json.load(open(os.path.join(os.path.dirname(L.__file__), "tune_db", "gfx950.json")))
        L.apply_tune_db()
        for logr, rows in db.get("pipeline", {}).get("min_rows", {}).items():
            assert L.pm_tune_get_pipeline_rows(int(logr)) == int(rows)
    finally:
        for r, v in before.items():
            L.pm_tune_set_pipeline_rows(r, v)
