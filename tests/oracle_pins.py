"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each ``pin_*`` function takes an ``oracle.Oracle`` instance and raises
``AssertionError`` on the first disagreement. They are run against the real
oracle (``test_oracle_pins.py``) and against copies of it with a planted
mistake (``test_oracle_planted.py``), so a dropped term, a wrong sign or index,
or a transposed operand anywhere in the oracle fails at least one of them.

None of these pins compares the oracle with itself: the expected values come
from Python integer arithmetic, from the independent brute force in
``oracle/bruteforce.py``, from closed forms, or from values the paper prints.
"""
from __future__ import annotations

import random

import numpy as np

from oracle import bruteforce as bf

Q60 = 0x0FFFFFFFFFFFC001          # 2^60 - 2^14 + 1
SMALL_PRIMES_1MOD128 = [257, 641, 769, 7681, 12289, 40961, 65537]


def _rand_poly(rng, n, q):
    return np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)


def _small_ntt_params(n):
    """A few (q, psi) with 2n | q-1, found by brute force in Python."""
    out = []
    for q in SMALL_PRIMES_1MOD128 + [Q60]:
        if (q - 1) % (2 * n):
            continue
        # brute-force psi of order exactly 2n: smallest g with g^n = -1
        for g in range(2, 5000):
            psi = pow(g, (q - 1) // (2 * n), q)
            if pow(psi, n, q) == q - 1:
                out.append((q, psi))
                break
    return out


# ---------------------------------------------------------------- Z_q ----

def pin_arith(o, trials=2000, seed=1):
    """or_mulmod/addmod/submod/powmod against Python integers (Sec. III Z_q)."""
    rng = random.Random(seed)
    moduli = [2, 3, 97, 2**31 - 1, Q60, 2**62 - 57, 2**63 + 29, 2**64 - 59]
    for q in moduli:
        edge = [0, 1, q - 1, q - 2 if q > 2 else 0, q // 2]
        pairs = [(a, b) for a in edge for b in edge]
        pairs += [(rng.randrange(q), rng.randrange(q)) for _ in range(trials // len(moduli))]
        for a, b in pairs:
            assert o.mulmod(a, b, q) == a * b % q, (a, b, q)
            assert o.addmod(a, b, q) == (a + b) % q, (a, b, q)
            assert o.submod(a, b, q) == (a - b) % q, (a, b, q)
        for _ in range(20):
            a, e = rng.randrange(q), rng.randrange(2**64)
            assert o.powmod(a, e, q) == pow(a, e, q)


def pin_barrett_worked_example(o, golden):
    """Sec. II-B worked example: the remainder is the textbook one."""
    a, b, q = golden["a"], golden["b"], golden["q"]
    assert o.mulmod(a, b, q) == (a * b) % q


# ------------------------------------------------------------ params ----

def pin_is_prime(o, seed=2):
    """or_is_prime against trial division (small n) and an independent
    Miller-Rabin (large n, including Carmichael numbers and prime squares)."""
    for n in range(0, 3000):
        assert o.is_prime(n) == bf.is_prime_trial(n), n
    rng = random.Random(seed)
    special = [561, 1105, 1729, 2465, 2821, 6601, 8911, 3215031751, 2**61 - 1,
               (2**31 - 1) ** 2, 4294967291 * 4294967279, Q60, 2**64 - 59]
    for n in special + [rng.randrange(2**40, 2**64) | 1 for _ in range(300)]:
        assert o.is_prime(n) == bf.is_prime_mr(n), n


def pin_ntt_primes(o, N, count, bits=60):
    """Primes q = 1 mod 2N below 2^bits, descending, none skipped (the prime
    rule for RNS limbs: the largest such primes below 2^60)."""
    got = o.ntt_primes(N, count, bits)
    assert len(got) == count
    two_n = 2 * N
    expect_top = ((2**bits - 2) // two_n) * two_n + 1
    cand = expect_top
    for q in got:
        assert q % two_n == 1 and q < 2**bits and bf.is_prime_mr(q), q
        # every candidate above q that was passed over must be composite
        while cand > q:
            assert not bf.is_prime_mr(cand), ("skipped prime", cand)
            cand -= two_n
        assert cand == q
        cand -= two_n


def pin_psi(o, q, N):
    """psi is a primitive 2N-th root of unity (psi^N = -1, psi^2N = 1), built
    from the smallest quadratic non-residue g (Euler's criterion)."""
    psi = o.find_psi(q, N)
    assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1
    g = next(g for g in range(2, 1000) if pow(g, (q - 1) // 2, q) == q - 1)
    assert psi == pow(g, (q - 1) // (2 * N), q)
    return psi


def pin_tables(o, q, N, psi):
    """psi_br[i] = psi^br(i), psi_inv_br[i] = psi^-br(i), br over log2 N bits."""
    fwd, inv = o.psi_tables(q, N, psi)
    bits = N.bit_length() - 1
    psi_inv = pow(psi, -1, q)
    for i in range(N):
        e = bf.bitrev(i, bits)
        assert int(fwd[i]) == pow(psi, e, q), i
        assert int(inv[i]) == pow(psi_inv, e, q), i
    if N >= 2:
        assert int(fwd[N // 2]) == psi and int(fwd[1]) ** 2 % q == q - 1
    return fwd, inv


# ------------------------------------------------------- polynomials ----

def pin_schoolbook_bruteforce(o, seed=3):
    """Schoolbook against the independent big-int expansion, N <= 64."""
    rng = random.Random(seed)
    for n in [1, 2, 4, 8, 16, 32, 64]:
        for q in [2, 17, 12289, Q60, 2**62 - 57]:
            a, b = _rand_poly(rng, n, q), _rand_poly(rng, n, q)
            assert [int(x) for x in o.polymul_schoolbook(a, b, q)] == bf.negacyclic(a, b, q), (n, q)


def pin_closed_forms(o):
    """N = 2 closed form and the monomial rule x^i x^j = +-x^((i+j) mod N)."""
    q = Q60
    for (a0, a1, b0, b1) in [(3, 5, 7, 11), (q - 1, q - 2, 1, q - 1), (0, 1, 0, 1)]:
        c = o.polymul_schoolbook([a0, a1], [b0, b1], q)
        assert int(c[0]) == (a0 * b0 - a1 * b1) % q and int(c[1]) == (a0 * b1 + a1 * b0) % q
    for n in [4, 16, 64]:
        for i in range(n):
            for j in range(0, n, 3):
                a = np.zeros(n, np.uint64); a[i] = 1
                b = np.zeros(n, np.uint64); b[j] = 1
                c = o.polymul_schoolbook(a, b, q)
                expect = np.zeros(n, np.uint64)
                expect[(i + j) % n] = 1 if i + j < n else q - 1
                assert np.array_equal(c, expect), (n, i, j)


def pin_ring_laws(o, seed=4):
    """Commutativity, distributivity and the identity on random inputs."""
    rng = random.Random(seed)
    q = Q60
    for n in [8, 32]:
        a, b, c = (_rand_poly(rng, n, q) for _ in range(3))
        ab, ba = o.polymul_schoolbook(a, b, q), o.polymul_schoolbook(b, a, q)
        assert np.array_equal(ab, ba)
        bc = np.array([(int(x) + int(y)) % q for x, y in zip(b, c)], np.uint64)
        lhs = o.polymul_schoolbook(a, bc, q)
        ac = o.polymul_schoolbook(a, c, q)
        rhs = np.array([(int(x) + int(y)) % q for x, y in zip(ab, ac)], np.uint64)
        assert np.array_equal(lhs, rhs)
        one = np.zeros(n, np.uint64); one[0] = 1
        assert np.array_equal(o.polymul_schoolbook(a, one, q), a)


def pin_ntt_eval(o, seed=5):
    """Alg. 5 output position p equals a(psi^(2 br(p)+1)): against the
    independent Python evaluation (N <= 64) and against the C brute-force
    evaluation (N <= 256, itself checked against Python at N <= 64)."""
    rng = random.Random(seed)
    for n in [2, 4, 8, 16, 32, 64]:
        for q, psi in _small_ntt_params(n):
            fwd, _ = o.psi_tables(q, n, psi)
            a = _rand_poly(rng, n, q)
            want = bf.ntt_by_evaluation(a, q, psi)
            assert [int(x) for x in o.ntt_fwd(a, q, fwd)] == want, (n, q)
            assert [int(x) for x in o.ntt_eval(a, q, psi)] == want, (n, q)
    for n in [128, 256]:
        q = Q60
        psi = o.find_psi(q, n)
        fwd, _ = o.psi_tables(q, n, psi)
        a = _rand_poly(rng, n, q)
        assert np.array_equal(o.ntt_fwd(a, q, fwd), o.ntt_eval(a, q, psi)), n


def pin_ntt_invariants(o, seed=6):
    """NTT(e0) = all ones, NTT(e1)[p] = psi^(2 br(p)+1), linearity."""
    rng = random.Random(seed)
    q = Q60
    for n in [16, 1024]:
        psi = o.find_psi(q, n)
        fwd, _ = o.psi_tables(q, n, psi)
        bits = n.bit_length() - 1
        e0 = np.zeros(n, np.uint64); e0[0] = 1
        assert np.all(o.ntt_fwd(e0, q, fwd) == 1)
        e1 = np.zeros(n, np.uint64); e1[1] = 1
        got = o.ntt_fwd(e1, q, fwd)
        for p in range(n):
            assert int(got[p]) == pow(psi, 2 * bf.bitrev(p, bits) + 1, q), (n, p)
        a, b = _rand_poly(rng, n, q), _rand_poly(rng, n, q)
        s = rng.randrange(q)
        lin = np.array([(int(x) + s * int(y)) % q for x, y in zip(a, b)], np.uint64)
        fa, fb, fl = o.ntt_fwd(a, q, fwd), o.ntt_fwd(b, q, fwd), o.ntt_fwd(lin, q, fwd)
        assert all(int(fl[i]) == (int(fa[i]) + s * int(fb[i])) % q for i in range(n))


def pin_ntt_roundtrip(o, sizes=(2, 8, 64, 1024, 2**13, 2**16), seed=7):
    """INTT(NTT(a)) = a and NTT(INTT(y)) = y."""
    rng = np.random.default_rng(seed)
    for n in sizes:
        q = o.ntt_primes(n, 1)[0]
        fwd, inv = o.psi_tables(q, n)
        a = (rng.integers(0, 2**62, n, dtype=np.uint64) % np.uint64(q)).astype(np.uint64)
        assert np.array_equal(o.ntt_inv(o.ntt_fwd(a, q, fwd), q, inv), a), n
        assert np.array_equal(o.ntt_fwd(o.ntt_inv(a, q, inv), q, fwd), a), n


def pin_psi_weighted_cyclic(o, seed=8):
    """The psi-weighted cyclic relation: a (*) b = psi^-i . (1/N) DFT_{w^-1}(
    DFT_w(psi^i . a) . DFT_w(psi^i . b)) with w = psi^2, written out with
    plain DFT sums in Python; equals the oracle's negacyclic product."""
    rng = random.Random(seed)
    for n in [4, 8, 16]:
        for q, psi in _small_ntt_params(n)[:3]:
            w = psi * psi % q
            a, b = _rand_poly(rng, n, q), _rand_poly(rng, n, q)
            pa = [int(a[i]) * pow(psi, i, q) % q for i in range(n)]
            pb = [int(b[i]) * pow(psi, i, q) % q for i in range(n)]
            dft = lambda v, r: [sum(v[i] * pow(r, i * j, q) for i in range(n)) % q for j in range(n)]
            h = [x * y % q for x, y in zip(dft(pa, w), dft(pb, w))]
            winv, ninv, psiinv = pow(w, -1, q), pow(n, -1, q), pow(psi, -1, q)
            c = [x * ninv % q for x in dft(h, winv)]
            c = [c[i] * pow(psiinv, i, q) % q for i in range(n)]
            assert [int(x) for x in o.polymul_schoolbook(a, b, q)] == c, (n, q)


def pin_polymul_ntt_vs_schoolbook(o, sizes=(2, 4, 16, 256, 1024, 4096), seed=9):
    """Eq. 1 path equals the schoolbook definition (N <= 2^12)."""
    rng = np.random.default_rng(seed)
    for n in sizes:
        for q in o.ntt_primes(n, 2):
            fwd, inv = o.psi_tables(q, n)
            a = (rng.integers(0, 2**62, n, dtype=np.uint64) % np.uint64(q)).astype(np.uint64)
            b = (rng.integers(0, 2**62, n, dtype=np.uint64) % np.uint64(q)).astype(np.uint64)
            assert np.array_equal(o.polymul_ntt(a, b, q, fwd, inv), o.polymul_schoolbook(a, b, q)), (n, q)


def pin_polymul_large(o, sizes=(2**16, 2**17), seed=10, coeffs=16, points=4):
    """Large N: sampled coefficients against the O(N) definition and the
    evaluation identity c(psi^(2j+1)) = a(psi^(2j+1)) b(psi^(2j+1)) (Horner)."""
    rng = np.random.default_rng(seed)
    for n in sizes:
        q = o.ntt_primes(n, 1)[0]
        psi = o.find_psi(q, n)
        fwd, inv = o.psi_tables(q, n, psi)
        a = (rng.integers(0, 2**62, n, dtype=np.uint64) % np.uint64(q)).astype(np.uint64)
        b = (rng.integers(0, 2**62, n, dtype=np.uint64) % np.uint64(q)).astype(np.uint64)
        c = o.polymul_ntt(a, b, q, fwd, inv)
        ks = [0, 1, n // 2, n - 1] + [int(k) for k in rng.integers(0, n, coeffs)]
        for k in ks:
            want = sum(int(a[i]) * int(b[k - i]) for i in range(k + 1)) - \
                sum(int(a[i]) * int(b[k + n - i]) for i in range(k + 1, n))
            assert int(c[k]) == want % q, (n, k)
        for j in [int(x) for x in rng.integers(0, n, points)]:
            pt = pow(psi, 2 * j + 1, q)
            assert o.poly_eval(c, q, pt) == o.poly_eval(a, q, pt) * o.poly_eval(b, q, pt) % q


def pin_coeff(o, seed=11):
    """or_polymul_coeff (one coefficient, O(N)) against the big-int expansion."""
    rng = random.Random(seed)
    for n in [1, 2, 8, 64]:
        q = Q60
        a, b = _rand_poly(rng, n, q), _rand_poly(rng, n, q)
        full = bf.negacyclic(a, b, q)
        for k in range(n):
            assert o.polymul_coeff(a, b, q, k) == full[k]


def pin_eval(o, seed=12):
    """Horner evaluation against term-by-term evaluation."""
    rng = random.Random(seed)
    for n in [1, 5, 64]:
        q = Q60
        a = _rand_poly(rng, n, q)
        for _ in range(5):
            x = rng.randrange(q)
            assert o.poly_eval(a, q, x) == bf.eval_poly(a, x, q)


ALL_FAST = [pin_arith, pin_is_prime, pin_schoolbook_bruteforce, pin_closed_forms,
            pin_ring_laws, pin_ntt_eval, pin_ntt_invariants, pin_psi_weighted_cyclic,
            pin_coeff, pin_eval]


def pin_mulmod_vec(o, seed=13):
    """Elementwise product against Python integers."""
    rng = random.Random(seed)
    for q in [3, 12289, Q60, 2**62 - 57]:
        a = [rng.randrange(q) for _ in range(200)] + [q - 1, 0, 1]
        b = [rng.randrange(q) for _ in range(200)] + [q - 1, q - 1, q - 1]
        got = o.mulmod_vec(np.array(a, np.uint64), np.array(b, np.uint64), q)
        assert [int(x) for x in got] == [x * y % q for x, y in zip(a, b)]


ALL_FAST.append(pin_mulmod_vec)
