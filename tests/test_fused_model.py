"""The fused polynomial multiplication (Sec. III-B, Alg. 7 and 8) modelled in
pure Python, pinned to the plain definition of the negacyclic product.

Pins: Alg. 7 equals its definition (last CT butterflies, product, halved
first GS butterfly) and the closed form (a0 b0 + alpha^2 a1 b1,
a0 b1 + a1 b0); the squared last-stage twiddles are the second-to-last
stage's up to the sign (-1)^i; Alg. 8 with the first GS stage omitted equals
schoolbook; the text's literal loop change (which omits the last GS stage)
does not.
"""
import random

import pytest

from oracle import bruteforce as BF
from oracle import fused_model as F


def _largest_prime(bits, two_n):
    q = ((1 << bits) - 1) // two_n * two_n + 1
    while not BF.is_prime_mr(q):
        q -= two_n
    return q


# (q, largest N with 2N | q - 1 that the tests use)
PRIMES = [(257, 64), (7681, 64), (12289, 64), (0x0FFFFFFFFFFFC001, 64), (_largest_prime(62, 128), 64)]


def _psi(q, n):
    g = 2
    while pow(g, (q - 1) // 2, q) != q - 1:
        g += 1
    psi = pow(g, (q - 1) // (2 * n), q)
    assert pow(psi, n, q) == q - 1
    return psi


def _rand_poly(rng, n, q):
    return [rng.randrange(q) for _ in range(n)]


def test_primes_fit():
    for q, nmax in PRIMES:
        assert BF.is_prime_mr(q) and (q - 1) % (2 * nmax) == 0


@pytest.mark.parametrize("q", [257, 12289, 0x0FFFFFFFFFFFC001])
def test_fused_pair_matches_definition(q):
    rng = random.Random(q)
    for _ in range(200):
        a0, a1, b0, b1 = (rng.randrange(q) for _ in range(4))
        alpha = rng.randrange(1, q)
        got = F.fused_pair(a0, a1, b0, b1, alpha * alpha % q, q)
        assert got == F.fused_pair_reference(a0, a1, b0, b1, alpha, q)
        assert got == ((a0 * b0 + alpha * alpha * a1 * b1) % q, (a0 * b1 + a1 * b0) % q)


@pytest.mark.parametrize("q,n", [(257, 64), (12289, 64), (0x0FFFFFFFFFFFC001, 64)])
def test_squared_last_stage_twiddles(q, n):
    psi_br, _ = F.tables(q, n, _psi(q, n))
    for i in range(n // 2):
        sq = psi_br[n // 2 + i] ** 2 % q
        want = psi_br[n // 4 + i // 2]
        assert sq == (want if i % 2 == 0 else (q - want) % q)


@pytest.mark.parametrize("q,nmax", PRIMES)
def test_fused_polymul_first_stage_reading_matches_schoolbook(q, nmax):
    rng = random.Random(nmax * 7 + q % 1000)
    n = 4
    while n <= nmax:
        psi_br, psi_inv_br = F.tables(q, n, _psi(q, n))
        for _ in range(3):
            a, b = _rand_poly(rng, n, q), _rand_poly(rng, n, q)
            assert F.polymul_fused(a, b, q, psi_br, psi_inv_br, "first") == BF.negacyclic(a, b, q), (q, n)
        n *= 2


@pytest.mark.parametrize("n", [8, 16, 64])
def test_literal_last_stage_reading_fails(n):
    """Omitting the last GS stage (the text's loop condition) does not give the product."""
    q = 12289
    psi_br, psi_inv_br = F.tables(q, n, _psi(q, n))
    rng = random.Random(n)
    a, b = _rand_poly(rng, n, q), _rand_poly(rng, n, q)
    assert F.polymul_fused(a, b, q, psi_br, psi_inv_br, "last") != BF.negacyclic(a, b, q)


def test_fused_monomials():
    """x^i * x^j = +-x^((i+j) mod N), the sign flipping exactly when i + j >= N."""
    q, n = 7681, 16
    psi_br, psi_inv_br = F.tables(q, n, _psi(q, n))
    for i in range(n):
        for j in range(n):
            a = [0] * n
            b = [0] * n
            a[i] = 1
            b[j] = 1
            c = F.polymul_fused(a, b, q, psi_br, psi_inv_br)
            want = [0] * n
            want[(i + j) % n] = 1 if i + j < n else q - 1
            assert c == want
