"""The LDS-poisoning debug build (libpm_poison.so: PM_POISON_LDS=1, every LDS
exchange first fills the row's LDS with words above every modulus) gives
bit-exact oracle results: no row kernel reads an LDS slot that the current
exchange did not write (a missing barrier or an indexing error would show up
as a mismatch). Called through the debug library's own C ABI, for every
row mode and both row geometries, single- and two-pass splits, the four-word
column pass from 2^4 to 2^7 rows (odd and even depths), the batched-jobs
kernels in both forms, and the software-pipelined product (row workgroups
beside column workgroups in one launch) for Eq. 2, the fused product and
squaring."""
import ctypes
import os

import numpy as np
import pytest

from gpu_helpers import first_mismatch, operands, oracle_ntt_fwd, oracle_ntt_inv, oracle_polymul, oracle_tables

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POISON = os.path.join(ROOT, "paper_2209_01290_amd", "libpm_poison.so")


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    assert os.path.exists(POISON), "libpm_poison.so is not built (python -m paper_2209_01290_amd.build --variant poison)"
    P = ctypes.CDLL(POISON)
    vp, sz, u64p = ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64)
    for name in ("pm_polymul", "pm_polymul_fused"):
        getattr(P, name).argtypes = [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp, vp]
    for name in ("pm_ntt_fwd", "pm_ntt_inv"):
        getattr(P, name).argtypes = [vp, sz, sz, sz, u64p, vp, vp]
    P.pm_tune_set_small.argtypes = [ctypes.c_int, ctypes.c_uint, ctypes.c_uint, ctypes.c_uint]
    P.pm_tune_set_small_batch.argtypes = [sz]
    P.pm_tune_set_pipeline.argtypes = [ctypes.c_int]
    P.pm_tune_set_jobs_pipeline.argtypes = [ctypes.c_int]
    P.pm_polymul_jobs.argtypes = [ctypes.POINTER(lib.Job), sz, vp, sz, vp]
    P.pm_polymul_jobs_workspace_bytes.argtypes = [ctypes.POINTER(lib.Job), sz]
    P.pm_polymul_jobs_workspace_bytes.restype = sz
    P.pm_last_error.restype = ctypes.c_char_p
    return lib, P


def _check(P, rc, what):
    assert rc == 0, "%s: %s" % (what, P.pm_last_error().decode())


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("geo", ["16-word", "4-word", "4-word-deep"])
@pytest.mark.parametrize("log2n", [6, 10, 12, 13, 14, 16])
def test_poisoned_lds_parity(env, log2n, geo):
    import torch
    L, P = env
    N, limbs, polys = 1 << log2n, 2, 2
    qs = L.pm_ntt_primes(N, limbs)
    prm = L.Params(N, limbs, primes=qs)
    fw_o, iv_o = oracle_tables(qs, N)
    a, b = operands(N, qs, polys, request=2500 + log2n)
    want = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    qarr = (ctypes.c_uint64 * limbs)(*qs)
    small = geo != "16-word"
    try:
        if small:
            if geo == "4-word":
                logc = log2n if log2n <= 12 else max(8, log2n - 4)
            else:
                # the deepest column pass: 2^7 rows, or rows of 2^5 words
                logc = max(5, log2n - 7)
                if log2n - logc < 2:
                    pytest.skip("no four-word column pass for N = 2^%d" % log2n)
            for op in (0, 1, 2):
                _check(P, P.pm_tune_set_small(op, log2n, min(logc, 12), 4), "tune")
            P.pm_tune_set_small_batch(1 << 22)
        nbytes = L.pm_polymul_workspace_bytes(N, limbs, polys) if not small else N * limbs * polys * 8
        ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device="cuda")
        da, db = L.to_device(a), L.to_device(b)
        for fn in ("pm_polymul", "pm_polymul_fused"):
            dc = torch.zeros_like(da)
            _check(P, getattr(P, fn)(da.data_ptr(), db.data_ptr(), dc.data_ptr(), N, limbs, polys, qarr,
                                     prm.psi_br.data_ptr(), prm.psi_inv_br.data_ptr(), ws.data_ptr(), _stream()), fn)
            torch.cuda.synchronize()
            msg = first_mismatch(L.to_host(dc).reshape(a.shape), want)
            assert msg is None, "%s N=%d: %s" % (fn, N, msg)
        sq = torch.zeros_like(da)          # squaring rows (a = b)
        _check(P, P.pm_polymul(da.data_ptr(), da.data_ptr(), sq.data_ptr(), N, limbs, polys, qarr,
                               prm.psi_br.data_ptr(), prm.psi_inv_br.data_ptr(), None, _stream()), "square")
        x = da.clone()
        _check(P, P.pm_ntt_fwd(x.data_ptr(), N, limbs, polys, qarr, prm.psi_br.data_ptr(), _stream()), "fwd")
        torch.cuda.synchronize()
        assert first_mismatch(L.to_host(sq).reshape(a.shape), oracle_polymul(a, a, qs, N, fw_o, iv_o)) is None
        assert first_mismatch(L.to_host(x).reshape(a.shape), oracle_ntt_fwd(a, qs, fw_o)) is None
        y = da.clone()
        _check(P, P.pm_ntt_inv(y.data_ptr(), N, limbs, polys, qarr, prm.psi_inv_br.data_ptr(), _stream()), "inv")
        torch.cuda.synchronize()
        assert first_mismatch(L.to_host(y).reshape(a.shape), oracle_ntt_inv(a, qs, iv_o)) is None
    finally:
        for op in (0, 1, 2):
            P.pm_tune_set_small(op, log2n, 0, 0)
        P.pm_tune_set_small_batch(0)


@pytest.mark.parametrize("log2n", [15, 16, 17])
def test_poisoned_lds_pipelined(env, log2n):
    """The software-pipelined product (pm_tune_set_pipeline(2): rows of one
    chunk beside the column passes of its neighbours in one launch) for
    Eq. 2, the fused product and squaring, through the debug library."""
    import torch
    L, P = env
    N, limbs, polys = 1 << log2n, 3, 2
    qs = L.pm_ntt_primes(N, limbs)
    prm = L.Params(N, limbs, primes=qs)
    fw_o, iv_o = oracle_tables(qs, N)
    a, b = operands(N, qs, polys, request=2700 + log2n)
    want = oracle_polymul(a, b, qs, N, fw_o, iv_o)
    want_sq = oracle_polymul(a, a, qs, N, fw_o, iv_o)
    qarr = (ctypes.c_uint64 * limbs)(*qs)
    ws = torch.empty(N * limbs * polys, dtype=torch.int64, device="cuda")
    da, db = L.to_device(a), L.to_device(b)
    P.pm_tune_set_pipeline(2)
    try:
        for fn, bp, w in (("pm_polymul", db, want), ("pm_polymul_fused", db, want), ("pm_polymul", da, want_sq)):
            dc = torch.zeros_like(da)
            _check(P, getattr(P, fn)(da.data_ptr(), bp.data_ptr(), dc.data_ptr(), N, limbs, polys, qarr,
                                     prm.psi_br.data_ptr(), prm.psi_inv_br.data_ptr(), ws.data_ptr(), _stream()), fn)
            torch.cuda.synchronize()
            msg = first_mismatch(L.to_host(dc).reshape(a.shape), w)
            assert msg is None, "%s%s N=%d: %s" % (fn, " (a = b)" if bp is da else "", N, msg)
    finally:
        P.pm_tune_set_pipeline(-1)


@pytest.mark.parametrize("chunks", [0, 3], ids=["three-pass", "pipelined"])
def test_poisoned_lds_jobs(env, chunks):
    """Mixed sizes through the batched-jobs row kernels (rows of 2^12, and
    whole small polynomials packed into one row task), as three launches and
    as the software-pipelined launches."""
    import torch
    L, P = env
    P.pm_tune_set_jobs_pipeline(chunks)
    jobs, keep, checks = [], [], []
    for log2n in (5, 9, 12, 14, 16, 17):
        N = 1 << log2n
        qs = L.pm_ntt_primes(N, 1)
        prm = L.Params(N, 1, primes=qs)
        a, b = operands(N, qs, 3, request=2600 + log2n)
        da, db = L.to_device(a[0]), L.to_device(b[0])
        dc = torch.zeros_like(da)
        jobs.append(L.make_job(log2n, 3, qs[0], prm.psi_br[0], prm.psi_inv_br[0], da, db, dc))
        keep += [prm, da, db, dc]
        checks.append((a, b, qs, N, dc))
    arr = (L.Job * len(jobs))(*jobs)
    try:
        need = P.pm_polymul_jobs_workspace_bytes(arr, len(jobs))
        ws = torch.empty(need // 8 + 64, dtype=torch.int64, device="cuda")
        _check(P, P.pm_polymul_jobs(arr, len(jobs), ws.data_ptr(), ws.numel() * 8, _stream()), "jobs")
        torch.cuda.synchronize()
    finally:
        P.pm_tune_set_jobs_pipeline(-1)
    for a, b, qs, N, dc in checks:
        fw, iv = oracle_tables(qs, N)
        msg = first_mismatch(L.to_host(dc).reshape(a.shape), oracle_polymul(a, b, qs, N, fw, iv))
        assert msg is None, "jobs N=%d: %s" % (N, msg)
