"""Drives every host-only path of the C ABI (no kernel is launched): argument
validation of each entry point, the parameter helpers, the tuning tables and
the job-table layout over many random job lists. Run under AddressSanitizer
by test_host_asan.py (argv[1] = the instrumented library)."""
import ctypes
import random
import sys

L = ctypes.CDLL(sys.argv[1])
vp, sz, u64, u32, i32, uint = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint
u64p, u32p = ctypes.POINTER(u64), ctypes.POINTER(u32)
L.pm_last_error.restype = ctypes.c_char_p
L.pm_ntt_primes.restype = sz
L.pm_ntt_primes.argtypes = [u64, uint, sz, u64p]
L.pm_find_psi.restype = u64
L.pm_find_psi.argtypes = [u64, sz]
L.pm_make_tables.argtypes = [u64, sz, u64, u64p, u64p]
L.pm_make_tables_u32.argtypes = [u32, sz, u32, u32p, u32p]
for f in ("pm_polymul", "pm_polymul_fused", "pm_polymul_stagewise", "pm_polymul_il"):
    getattr(L, f).argtypes = [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp, vp]
for f in ("pm_polymul_u32", "pm_polymul_fused_u32"):
    getattr(L, f).argtypes = [vp, vp, vp, sz, sz, sz, u32p, vp, vp, vp, vp]
for f in ("pm_ntt_fwd", "pm_ntt_inv", "pm_ntt_fwd_il", "pm_ntt_inv_il"):
    getattr(L, f).argtypes = [vp, sz, sz, sz, u64p, vp, vp]
for f in ("pm_ntt_fwd_u32", "pm_ntt_inv_u32"):
    getattr(L, f).argtypes = [vp, sz, sz, sz, u32p, vp, vp]
for f in ("pm_polymul_workspace_bytes", "pm_polymul_u32_workspace_bytes", "pm_polymul_il_workspace_bytes",
          "pm_polymul_stagewise_workspace_bytes"):
    getattr(L, f).argtypes = [sz, sz, sz]
    getattr(L, f).restype = sz
L.pm_barrett_mulmod.argtypes = [vp, vp, vp, sz, u64, vp]
L.pm_tune_set.argtypes = [i32, uint, uint]
L.pm_tune_get.argtypes = [i32, uint]
L.pm_tune_set_small.argtypes = [i32, uint, uint, uint]
L.pm_tune_get_small.argtypes = [i32, uint, ctypes.POINTER(uint), ctypes.POINTER(uint)]
L.pm_tune_set_small_batch.argtypes = [sz]
L.pm_tune_get_small_batch.restype = sz
L.pm_tune_set_small_limit.argtypes = [i32, uint, sz]
L.pm_tune_get_small_limit.argtypes = [i32, uint]
L.pm_tune_get_small_limit.restype = sz


class Job(ctypes.Structure):
    _fields_ = [("log2n", u32), ("count", u32), ("q", u64), ("psi_br", vp), ("psi_inv_br", vp),
                ("a", vp), ("b", vp), ("c", vp)]


L.pm_polymul_jobs_workspace_bytes.argtypes = [ctypes.POINTER(Job), sz]
L.pm_polymul_jobs_workspace_bytes.restype = sz
L.pm_polymul_jobs.argtypes = [ctypes.POINTER(Job), sz, vp, sz, vp]
L.pm_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Job), sz, uint]
EINVAL = -1
F = vp(0x10000)
rng = random.Random(7)


def primes(N, n, bits=60):
    out = (u64 * n)()
    got = L.pm_ntt_primes(2 * N, bits, n, out)
    return [int(out[i]) for i in range(got)]


# parameter helpers
for N in (2, 16, 1024, 1 << 17):
    qs = primes(N, 3)
    assert len(qs) == 3
    psi = L.pm_find_psi(qs[0], N)
    if N <= 1024:
        f, i = (u64 * N)(), (u64 * N)()
        assert L.pm_make_tables(qs[0], N, psi, f, i) == 0
        assert L.pm_make_tables(qs[0], N, 1, f, i) == EINVAL          # 1^N != q - 1
q30 = primes(1024, 1, 30)[0]
f32, i32a = (u32 * 1024)(), (u32 * 1024)()
assert L.pm_make_tables_u32(q30, 1024, L.pm_find_psi(q30, 1024), f32, i32a) == 0
assert L.pm_ntt_primes(0, 60, 4, (u64 * 4)()) == 0

# validation of every entry point (returns before any device work)
q = (u64 * 1)(primes(1024, 1)[0])
qb = (u64 * 1)(q[0] + 2)
q32 = (u32 * 1)(q30)
for N in (0, 1, 3, 1000, 1 << 18):
    for f in ("pm_polymul", "pm_polymul_fused", "pm_polymul_stagewise", "pm_polymul_il"):
        assert getattr(L, f)(F, F, F, N, 1, 1, q, F, F, F, None) == EINVAL
    for f in ("pm_ntt_fwd", "pm_ntt_inv", "pm_ntt_fwd_il", "pm_ntt_inv_il"):
        assert getattr(L, f)(F, N, 1, 1, q, F, None) == EINVAL
    for f in ("pm_polymul_u32", "pm_polymul_fused_u32"):
        assert getattr(L, f)(F, F, F, N, 1, 1, q32, F, F, F, None) == EINVAL
    assert L.pm_ntt_fwd_u32(F, N, 1, 1, q32, F, None) == EINVAL
    assert len(L.pm_last_error()) > 0
assert L.pm_polymul(F, F, F, 1024, 1, 1, qb, F, F, F, None) == EINVAL
assert L.pm_polymul(vp(0x10004), F, F, 1024, 1, 1, q, F, F, F, None) == EINVAL
assert L.pm_polymul(F, F, F, 1024, 0, 1, q, F, F, F, None) == EINVAL
assert L.pm_polymul(F, F, F, 1024, 1, 70000, q, F, F, F, None) == EINVAL
assert L.pm_polymul(F, F, F, 1024, 1, 1, None, F, F, F, None) == EINVAL
many = (u64 * 200)(*([q[0]] * 199 + [q[0] + 1]))
assert L.pm_polymul(F, F, F, 1024, 200, 1, many, F, F, F, None) == EINVAL   # last limb even
assert L.pm_barrett_mulmod(F, F, F, 0, 97, None) == EINVAL
for n in range(1, 18):
    for f in ("pm_polymul_workspace_bytes", "pm_polymul_u32_workspace_bytes", "pm_polymul_il_workspace_bytes"):
        getattr(L, f)(1 << n, 3, 5)

# tuning tables
for op in (0, 1, 2):
    for n in range(0, 20):
        for c in range(0, 16):
            L.pm_tune_set(op, n, c)
            for w in (0, 4, 8, 16):
                L.pm_tune_set_small(op, n, c, w)
        L.pm_tune_get(op, n)
        a, b = uint(), uint()
        L.pm_tune_get_small(op, n, ctypes.byref(a), ctypes.byref(b))
        L.pm_tune_set(op, n, 0) if 1 <= n <= 17 else None
        L.pm_tune_set_small(op, n, 0, 0)
        L.pm_tune_set_small_limit(op, n, 1 << 20)
        L.pm_tune_get_small_limit(op, n)
        L.pm_tune_set_small_limit(op, n, 0)
assert L.pm_tune_get_small(5, 3, None, None) == EINVAL
L.pm_tune_set_small_batch(1 << 20)
assert L.pm_tune_get_small_batch() == 1 << 20
L.pm_tune_set_small_batch(0)

# job-table layout over random job lists (sizes only; no launch)
pq = {n: primes(1 << n, 4) for n in range(1, 18)}
for trial in range(3000):
    nj = rng.randint(1, 40)
    jobs = (Job * nj)()
    bad = rng.random() < 0.3
    for j in range(nj):
        n = rng.randint(1, 17)
        base = 0x100000 * (j + 1)
        jobs[j] = Job(n, rng.randint(1, 5), pq[n][rng.randint(0, 3)], base, base + 0x1000,
                      base + 0x2000, base + (0x2000 if rng.random() < 0.2 else 0x3000), base + 0x4000)
    if bad:
        k = rng.randrange(nj)
        which = rng.randint(0, 4)
        if which == 0:
            jobs[k].log2n = rng.choice([0, 18, 40])
        elif which == 1:
            jobs[k].count = 0
        elif which == 2:
            jobs[k].q = jobs[k].q + 1
        elif which == 3:
            jobs[k].a = 0
        else:
            jobs[k].c = jobs[k].c + 4
    need = L.pm_polymul_jobs_workspace_bytes(jobs, nj)
    assert (need == 0) == bad, (trial, bad, need)
    if bad:
        assert L.pm_polymul_jobs(jobs, nj, vp(0x1000000), 1 << 40, None) == EINVAL
        p = vp()
        assert L.pm_plan_create(ctypes.byref(p), jobs, nj, 0) == EINVAL and not p.value
assert L.pm_polymul_jobs_workspace_bytes(None, 0) == 0
print("host paths ok")
