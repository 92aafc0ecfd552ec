"""Batched job tables (pm_polymul_jobs, pm_plan_*): mixed N, moduli and
aliasing in one batch, checked word for word against the oracle; graph
replays checked one by one with eager work in between. Both forms: three
launches (one per pass of Eq. 2) and the software-pipelined launches (rows of
2^12 words of one chunk of products beside the column passes of its
neighbours), with chunk boundaries inside jobs, empty chunks, and the
automatic choice at a batch above the pipelining threshold."""
import numpy as np
import pytest

from gpu_helpers import first_mismatch, oracle_polymul, oracle_tables
from paper_2209_01290_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    yield lib
    lib.pm_tune_set_jobs_pipeline(-1)


# (log2n, count, bits of the prime search, prime index, alias)
MIX = [(1, 3, 60, 0, ""), (4, 2, 60, 1, "c=a"), (8, 5, 30, 0, ""), (10, 4, 60, 2, "c=b"),
       (12, 3, 60, 0, ""), (13, 2, 62, 0, "a=b"), (14, 2, 60, 3, ""), (15, 1, 61, 0, "c=a"),
       (16, 3, 60, 1, "c=b"), (17, 2, 60, 0, ""), (16, 1, 35, 0, "a=b=c"), (11, 7, 60, 4, "")]


def _build(L, mix, request0=0):
    import torch
    jobs, keep, want = [], [], []
    for i, (log2n, count, bits, qi, alias) in enumerate(mix):
        N = 1 << log2n
        q = L.pm_ntt_primes(N, qi + 1, bits)[qi]
        a, b = synth.operands(synth.SEED_BASE + 4, [q], count, N, request=request0 + i)
        if "a=b" in alias:
            b = a.copy()
        fw_o, iv_o = oracle_tables([q], N)
        want.append(oracle_polymul(a, b, [q], N, fw_o, iv_o)[0])
        fw, iv = L.pm_make_tables(q, N)
        dfw, div = L.to_device(fw), L.to_device(iv)
        da = L.to_device(a[0])
        db = da if "a=b" in alias else L.to_device(b[0])
        if alias == "c=a" or alias == "a=b=c":
            dc = da
        elif alias == "c=b":
            dc = db
        else:
            dc = torch.empty_like(da)
        jobs.append(L.make_job(log2n, count, q, dfw, div, da, db, dc))
        keep.append((dfw, div, da, db, dc, a, b))
    return jobs, keep, want


def _check_all(L, keep, want, what):
    for i, (k, w) in enumerate(zip(keep, want)):
        got = L.to_host(k[4]).reshape(w.shape)
        msg = first_mismatch(got, w)
        assert msg is None, "%s job %d (N=2^%d): %s" % (what, i, MIX[i][0] if i < len(MIX) else -1, msg)


def test_jobs_one_shot(L):
    import torch
    jobs, keep, want = _build(L, MIX)
    nbytes = L.pm_polymul_jobs_workspace_bytes(jobs)
    assert nbytes > 0
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
    L.pm_polymul_jobs(jobs, ws)
    torch.cuda.synchronize()
    _check_all(L, keep, want, "one-shot")


@pytest.mark.parametrize("flags", [0, 1], ids=["graph", "direct"])
def test_plan_replays(L, flags):
    """A plan replayed several times, with eager library work and host
    synchronization between replays; every replay is checked."""
    import torch
    jobs, keep, want = _build(L, MIX, request0=50)
    plan = L.pm_plan_create(jobs, flags)
    try:
        assert L.pm_plan_device_bytes(plan) > 0
        for rep in range(3):
            # restore the inputs that the previous replay overwrote (aliased outputs)
            for k in keep:
                k[2].copy_(L.to_device(k[5][0]))
                if k[3].data_ptr() != k[2].data_ptr():
                    k[3].copy_(L.to_device(k[6][0]))
            # unrelated eager work on the same stream between replays
            x = L.to_device(np.arange(1, 1025, dtype=np.uint64))
            L.pm_barrett_mulmod(x, x, x, 12289)
            torch.cuda.synchronize()
            L.pm_plan_launch(plan)
            torch.cuda.synchronize()
            _check_all(L, keep, want, "replay %d" % rep)
    finally:
        L.pm_plan_destroy(plan)


def test_plan_reads_new_inputs(L):
    """Buffers are read again at each launch: new operands give new products."""
    import torch
    mix = [(16, 2, 60, 0, ""), (12, 3, 60, 1, "")]
    jobs, keep, want = _build(L, mix, request0=90)
    plan = L.pm_plan_create(jobs)
    try:
        L.pm_plan_launch(plan)
        torch.cuda.synchronize()
        for k, w in zip(keep, want):
            assert first_mismatch(L.to_host(k[4]).reshape(w.shape), w) is None
        # new operands in the same buffers
        for i, (log2n, count, bits, qi, _) in enumerate(mix):
            N = 1 << log2n
            q = L.pm_ntt_primes(N, qi + 1, bits)[qi]
            a, b = synth.operands(synth.SEED_BASE + 5, [q], count, N, request=i)
            keep[i][2].copy_(L.to_device(a[0]))
            keep[i][3].copy_(L.to_device(b[0]))
            fw_o, iv_o = oracle_tables([q], N)
            want[i] = oracle_polymul(a, b, [q], N, fw_o, iv_o)[0]
        L.pm_plan_launch(plan)
        torch.cuda.synchronize()
        for k, w in zip(keep, want):
            assert first_mismatch(L.to_host(k[4]).reshape(w.shape), w) is None
    finally:
        L.pm_plan_destroy(plan)


def test_jobs_validation(L):
    import torch
    jobs, keep, _ = _build(L, [(10, 1, 60, 0, "")])
    bad = L.Job.from_buffer_copy(jobs[0])
    bad.q = bad.q + 2
    with pytest.raises(L.PMError):
        L.pm_plan_create([bad])
    ws = torch.empty(16, dtype=torch.int64, device="cuda")
    with pytest.raises(L.PMError):
        L.pm_polymul_jobs(jobs + [bad], ws)


def _launch_counts(L, fn):
    import torch
    L.pm_prof_enable(True)
    try:
        L.pm_prof_read()
        fn()
        torch.cuda.synchronize()
        return {name: n for name, (n, _ms) in L.pm_prof_read().items()}
    finally:
        L.pm_prof_enable(False)


# chunk counts: boundaries inside jobs of several products (2, 3, 7) and more
# chunks than pipelined products (40: empty chunks are skipped)
@pytest.mark.parametrize("chunks", [2, 3, 7, 40])
def test_jobs_pipelined(L, chunks):
    import torch
    jobs, keep, want = _build(L, MIX, request0=200 + chunks)
    L.pm_tune_set_jobs_pipeline(chunks)
    try:
        nbytes = L.pm_polymul_jobs_workspace_bytes(jobs)
        ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
        counts = _launch_counts(L, lambda: L.pm_polymul_jobs(jobs, ws))
    finally:
        L.pm_tune_set_jobs_pipeline(-1)
    _check_all(L, keep, want, "pipelined G=%d" % chunks)
    # the jobs of N >= 2^12 ran in pipelined launches (at most G + 2), the
    # smaller ones in one three-pass row launch (rows up to 2^11) before them
    assert 1 <= counts.get("jobs_pipe_mul_c12", 0) <= chunks + 2, counts
    assert counts.get("jobs_row_mul_c11", 0) == 1 and "jobs_col_fwd" not in counts, counts
    assert "jobs_row_mul_c12" not in counts, counts


def test_plan_replays_pipelined(L):
    """The pipelined launches captured in a plan's graph, replayed with eager
    work in between; every replay checked."""
    import torch
    jobs, keep, want = _build(L, MIX, request0=300)
    L.pm_tune_set_jobs_pipeline(3)
    try:
        plan = L.pm_plan_create(jobs)
    finally:
        L.pm_tune_set_jobs_pipeline(-1)
    try:
        for rep in range(3):
            for k in keep:
                k[2].copy_(L.to_device(k[5][0]))
                if k[3].data_ptr() != k[2].data_ptr():
                    k[3].copy_(L.to_device(k[6][0]))
            x = L.to_device(np.arange(1, 1025, dtype=np.uint64))
            L.pm_barrett_mulmod(x, x, x, 12289)
            torch.cuda.synchronize()
            L.pm_plan_launch(plan)
            torch.cuda.synchronize()
            _check_all(L, keep, want, "pipelined replay %d" % rep)
    finally:
        L.pm_plan_destroy(plan)


def test_jobs_pipelined_automatic_at_threshold(L):
    """Above 2048 rows of 2^12 words the default pipelines the table: the
    result equals the three-pass form word for word, and the oracle on
    sampled products of every job."""
    import torch
    from gpu_helpers import oracle_tables as ot
    import oracle
    # 40 x 2^16 (640 rows) + 44 x 2^17 (1408 rows) = 2048 rows, 4 jobs with chunk boundaries inside them
    spec = [(16, 25, 0), (17, 20, 1), (16, 15, 2), (17, 24, 3)]
    jobs, keep = [], []
    for i, (log2n, count, qi) in enumerate(spec):
        N = 1 << log2n
        q = L.pm_ntt_primes(N, qi + 1)[qi]
        a, b = synth.operands(synth.SEED_BASE + 6, [q], count, N, request=i)
        fw, iv = L.pm_make_tables(q, N)
        dfw, div = L.to_device(fw), L.to_device(iv)
        da, db = L.to_device(a[0]), L.to_device(b[0])
        dc = torch.empty_like(da)
        jobs.append(L.make_job(log2n, count, q, dfw, div, da, db, dc))
        keep.append((dfw, div, da, db, dc, a, b, q))
    nbytes = max(L.pm_polymul_jobs_workspace_bytes(jobs), 8)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
    L.pm_tune_set_jobs_pipeline(-1)
    counts = _launch_counts(L, lambda: L.pm_polymul_jobs(jobs, ws))
    assert counts.get("jobs_pipe_mul_c12", 0) == 4, counts          # G = 2: four launches
    piped = [L.to_host(k[4]).copy() for k in keep]
    for k in keep:
        k[4].zero_()
    L.pm_tune_set_jobs_pipeline(0)
    try:
        nbytes = max(L.pm_polymul_jobs_workspace_bytes(jobs), 8)
        ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
        counts = _launch_counts(L, lambda: L.pm_polymul_jobs(jobs, ws))
    finally:
        L.pm_tune_set_jobs_pipeline(-1)
    assert "jobs_pipe_mul_c12" not in counts and counts.get("jobs_col_fwd", 0) == 1, counts
    o = oracle.default()
    for i, k in enumerate(keep):
        three = L.to_host(k[4])
        assert np.array_equal(three, piped[i]), "job %d: pipelined and three-pass differ" % i
        log2n, count = spec[i][0], spec[i][1]
        q, a, b = k[7], k[5], k[6]
        fw, iv = ot([q], 1 << log2n)
        for p in (0, count // 2, count - 1):
            want = o.polymul_ntt(a[0, p], b[0, p], q, fw[0], iv[0])
            msg = first_mismatch(piped[i].reshape(count, -1)[p], want)
            assert msg is None, "job %d product %d: %s" % (i, p, msg)


@pytest.mark.parametrize("chunks", [0, 3])
def test_jobs_order_independent(L, chunks):
    """The work-item maps list jobs grouped by twiddle table, not in the
    caller's order: the same jobs given in another order (tables shared by
    several jobs of one size, sizes interleaved differently) produce the same
    words, in the three-pass and the pipelined form, and match the oracle."""
    import torch
    spec = []   # (log2n, count, prime index): three tables per size, each used by several jobs
    for r in range(3):
        for log2n in (12, 13, 15, 16, 17):
            for qi in (0, 1, 2):
                spec.append((log2n, 1 + (r + qi) % 2, qi))
    rng = np.random.default_rng(20901290)
    tables, jobs, keep = {}, [], []
    for i, (log2n, count, qi) in enumerate(spec):
        N = 1 << log2n
        if (log2n, qi) not in tables:
            q = L.pm_ntt_primes(N, qi + 1)[qi]
            fw, iv = L.pm_make_tables(q, N)
            tables[(log2n, qi)] = (q, L.to_device(fw), L.to_device(iv))
        q, dfw, div = tables[(log2n, qi)]
        a, b = synth.operands(synth.SEED_BASE + 8, [q], count, N, request=i)
        da, db = L.to_device(a[0]), L.to_device(b[0])
        keep.append([da, db, torch.empty_like(da), a, b, q, log2n, count])
        jobs.append((log2n, count, q, dfw, div))
    outs = []
    L.pm_tune_set_jobs_pipeline(chunks)
    try:
        for perm in (np.arange(len(spec)), rng.permutation(len(spec)), np.arange(len(spec))[::-1]):
            for k in keep:
                k[2].fill_(-1)
            job_list = [L.make_job(jobs[i][0], jobs[i][1], jobs[i][2], jobs[i][3], jobs[i][4],
                                   keep[i][0], keep[i][1], keep[i][2]) for i in perm]
            nbytes = max(L.pm_polymul_jobs_workspace_bytes(job_list), 8)
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
            L.pm_polymul_jobs(job_list, ws)
            torch.cuda.synchronize()
            outs.append([L.to_host(k[2]).copy() for k in keep])
    finally:
        L.pm_tune_set_jobs_pipeline(-1)
    for j in (1, 2):
        for i in range(len(spec)):
            assert np.array_equal(outs[0][i], outs[j][i]), "job %d differs between orders 0 and %d" % (i, j)
    import oracle
    o = oracle.default()
    for i in range(0, len(spec), 7):
        da, db, dc, a, b, q, log2n, count = keep[i]
        fw, iv = oracle_tables([q], 1 << log2n)
        want = o.polymul_ntt(a[0, count - 1], b[0, count - 1], q, fw[0], iv[0])
        msg = first_mismatch(outs[0][i].reshape(count, -1)[count - 1], want)
        assert msg is None, "job %d (N=2^%d): %s" % (i, log2n, msg)
