"""Models of Alg. 2, 3 and 4 (Sec. II-B) against the paper's statements.

Pins: the worked example (a=994674970, b=994705408, q=994705409), the bound of
at most one correctional subtraction for Alg. 4 (exhaustively for tiny moduli,
by sampling for 30- to 62-bit moduli), and the draft table of correction
counts for 30-bit moduli.
"""
import json
import os
import random

import pytest

from oracle import barrett_models as B

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_worked_example():
    g = _golden("barrett_worked_example.json")
    a, b, q = g["a"], g["b"], g["q"]
    x = a * b
    r2, k2 = B.classical(x, q, beta=32)
    r3, k3 = B.dhem_palisade(x, q, beta=34)
    r4, k4 = B.proposed(x, q, beta=32)
    assert r2 == r3 == r4 == x % q == 30439
    assert k2 == 2          # the classical reduction needs a second subtraction here
    assert k3 == 1 and k4 == 1


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7])
def test_proposed_at_most_one_correction_exhaustive(m):
    worst4 = worst2 = 0
    qs = range(2 ** (m - 1), 2 ** m) if m <= 6 else range(2 ** (m - 1) + 1, 2 ** m, 2)
    for q in qs:
        for x in range(2 ** (2 * m)):
            r, k = B.proposed(x, q)
            assert r == x % q
            worst4 = max(worst4, k)
            if m >= 2:
                r2, k2 = B.classical(x, q)
                assert r2 == x % q
                worst2 = max(worst2, k2)
    assert worst4 <= 1
    assert worst2 <= 2


@pytest.mark.parametrize("m", [30, 59, 60, 61, 62])
def test_proposed_at_most_one_correction_sampled(m):
    rng = random.Random(m)
    for _ in range(20000):
        q = rng.randrange(2 ** (m - 1) + 1, 2 ** m, 2)
        x = rng.randrange(2 ** (2 * m))
        r, k = B.proposed(x, q)
        assert r == x % q and k <= 1
    # products of canonical operands, the case the GPU path meets
    for _ in range(5000):
        q = rng.randrange(2 ** (m - 1) + 1, 2 ** m, 2)
        a, b = rng.randrange(q), rng.randrange(q)
        r, k = B.proposed(a * b, q)
        assert r == a * b % q and k <= 1


def test_correction_table_30bit():
    g = _golden("barrett_correction_table.json")
    rng = random.Random(2209)
    trials = 200000
    m = g["modulus_bits"]
    counts = {"classical_alg2": [0, 0, 0], "proposed_alg4": [0, 0, 0]}
    for _ in range(trials):
        q = rng.randrange(2 ** (m - 1) + 1, 2 ** m, 2)
        x = rng.randrange(2 ** (2 * m))
        counts["classical_alg2"][B.classical(x, q, beta=32)[1]] += 1
        counts["proposed_alg4"][B.proposed(x, q, beta=32)[1]] += 1
    tol = g["tolerance_percentage_points"]
    for name, want in g["percent_with_k_corrections"].items():
        got = [100.0 * c / trials for c in counts[name]]
        for k in range(3):
            assert abs(got[k] - want[k]) <= tol, (name, k, got, want)
