"""Models of the paper's Barrett reductions, in Python integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. II-B compares three reductions of x < 2^(2m) modulo q (m = len(q)). All
three are members of Dhem and Quisquater's generalised Barrett reduction,
which approximates the quotient floor(x / q) from two truncations:

    mu   = floor(2^(m + alpha) / q)                      precomputed per q
    quot = floor( floor(x / 2^(m + beta)) * mu / 2^(alpha - beta) )
    r    = x - quot * q, then subtract q while r >= q

Since x / q = (x / 2^(m + beta)) * (2^(m + alpha) / q) / 2^(alpha - beta),
dropping the two fractional parts can only make quot smaller, never larger,
so r >= 0; how much smaller (hence how many subtractions) depends on alpha
and beta. The paper's three reductions are the parameter choices

    classical  (Alg. 2, Barrett's original)  alpha = m,     beta = -1
    dhem_palisade (Alg. 3)                   alpha = m + 3, beta = -2
    proposed   (Alg. 4)                      alpha = m + 1, beta = -2

(the paper writes alpha relative to the modulus length, e.g. "N + 3"). The
word-size limit the paper states for each is asserted: len(q) <= word - 2
for Alg. 2 and Alg. 4, len(q) <= word - 4 for Alg. 3 (mu < 2^(alpha + 1)
and the values in between must be word-sized).

Each function returns ``(remainder, corrections)`` with ``corrections`` the
number of subtractions that were actually taken. The loop has no bound, so a
model never hides a case needing more corrections than its algorithm allows;
the tests check the counts against the bounds the paper states.
"""
from __future__ import annotations


def bitlen(a: int) -> int:
    """len(a) = floor(log2 a) + 1 (Sec. II, definition after Shoup)."""
    assert a > 0
    return a.bit_length()


def dq_constants(q: int, alpha_off: int, beta: int):
    """(m, mu, first shift, second shift) of the generalised reduction with
    alpha = m + alpha_off: mu = floor(2^(m + alpha) / q), x is truncated by
    m + beta bits and c * mu by alpha - beta bits."""
    m = bitlen(q)
    alpha = m + alpha_off
    return m, (1 << (m + alpha)) // q, m + beta, alpha - beta


def dq_reduce(x: int, q: int, alpha_off: int, beta: int):
    """x mod q by the generalised Barrett reduction; (remainder, corrections)."""
    m, mu, s1, s2 = dq_constants(q, alpha_off, beta)
    assert 0 <= x < 1 << (2 * m), "the reduction takes x < 2^(2m)"
    assert s1 >= 0, "modulus too short for this truncation"
    quot = ((x >> s1) * mu) >> s2
    r = x - quot * q
    assert r >= 0, "approximate quotient exceeded the true quotient"
    k = 0
    while r >= q:
        r -= q
        k += 1
    return r, k


# The paper's three instantiations: (alpha - m, beta) and the extra bits the
# word must hold beyond len(q) for mu to be word-sized (Sec. II-B: len(q) <=
# word - 2 for Alg. 2 and Alg. 4, len(q) <= word - 4 for Alg. 3).
CLASSICAL = (0, -1, 2)
DHEM_PALISADE = (3, -2, 4)
PROPOSED = (1, -2, 2)


def _variant(params, x, q, word):
    alpha_off, beta, headroom = params
    assert bitlen(q) <= word - headroom, "modulus too long for this variant's word size"
    return dq_reduce(x, q, alpha_off, beta)


def classical(x: int, q: int, beta: int = 64):
    """Alg. 2 (classical Barrett); `beta` is the word size in bits."""
    return _variant(CLASSICAL, x, q, beta)


def dhem_palisade(x: int, q: int, beta: int = 64):
    """Alg. 3 (Dhem-Quisquater, alpha = len(q) + 3, beta = -2)."""
    return _variant(DHEM_PALISADE, x, q, beta)


def proposed(x: int, q: int, beta: int = 64):
    """Alg. 4 (the paper's choice, alpha = len(q) + 1, beta = -2)."""
    return _variant(PROPOSED, x, q, beta)


def proposed_constants(q: int):
    """(m, mu, shift1, shift2) of Alg. 4 for modulus q."""
    return dq_constants(q, *PROPOSED[:2])
