"""Step-by-step models of the paper's Barrett reductions, in Python integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Each function follows one algorithm of Sec. II-B in the paper's own order and
notation and returns ``(remainder, corrections)`` where ``corrections`` counts
the correctional subtractions that were actually taken. Python integers are
unbounded, so the word-size conditions of the algorithms are asserted instead
of being enforced by overflow.

  classical(x, q)   Alg. 2: mu = floor(2^(2m)/q), c = x >> (m-1),
                    quot = (c*mu) >> (m+1), up to two subtractions.
  dhem_palisade     Alg. 3: Dhem-Quisquater with alpha = N+3, beta = -2:
                    mu = floor(2^(2m+3)/q), c = x >> (m-2), quot = (c*mu) >> (m+5).
  proposed(x, q)    Alg. 4: Dhem-Quisquater with alpha = N+1, beta = -2:
                    mu = floor(2^(2m+1)/q), c = x >> (m-2), quot = (c*mu) >> (m+3).

The loops are written with a generic ``while r >= q`` so that a model never
hides a case needing more corrections than its algorithm allows; tests check
the counts against the bounds the paper states.
"""
from __future__ import annotations


def bitlen(a: int) -> int:
    """len(a) = floor(log2 a) + 1 (Sec. II, definition after Shoup)."""
    assert a > 0
    return a.bit_length()


def _finish(x: int, quot: int, q: int):
    r = x - quot * q
    assert r >= 0, "approximate quotient exceeded the true quotient"
    k = 0
    while r >= q:
        r -= q
        k += 1
    return r, k


def classical(x: int, q: int, beta: int = 64):
    m = bitlen(q)
    assert m <= beta - 2 and 0 <= x < 2 ** (2 * m)
    mu = (2 ** (2 * m)) // q
    c = x >> (m - 1)
    quot = (c * mu) >> (m + 1)
    return _finish(x, quot, q)


def dhem_palisade(x: int, q: int, beta: int = 64):
    m = bitlen(q)
    assert m <= beta - 4 and 0 <= x < 2 ** (2 * m)
    mu = (2 ** (2 * m + 3)) // q
    c = x >> (m - 2)
    quot = (c * mu) >> (m + 5)
    return _finish(x, quot, q)


def proposed(x: int, q: int, beta: int = 64):
    m = bitlen(q)
    assert 2 <= m <= beta - 2 and 0 <= x < 2 ** (2 * m)
    mu = (2 ** (2 * m + 1)) // q
    c = x >> (m - 2)
    quot = (c * mu) >> (m + 3)
    return _finish(x, quot, q)


def proposed_constants(q: int):
    """(m, mu, shift1, shift2) of Alg. 4 for modulus q."""
    m = bitlen(q)
    return m, (2 ** (2 * m + 1)) // q, m - 2, m + 3
