"""The CPU oracle against what the paper and the mathematics fix.

These tests gate every parity claim: the GPU library is compared with the
oracle, so the oracle is first pinned to closed forms, independent brute force,
invariants of the transform and the paper's printed values.
"""
import json
import os

import pytest

import oracle_pins as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("pin", P.ALL_FAST, ids=lambda f: f.__name__)
def test_fast_pin(orc, pin):
    pin(orc)


def test_barrett_worked_example(orc):
    P.pin_barrett_worked_example(orc, _golden("barrett_worked_example.json"))


@pytest.mark.parametrize("N,count", [(1024, 1), (2**14, 32), (2**16, 48), (2**17, 60)])
def test_ntt_primes(orc, N, count):
    P.pin_ntt_primes(orc, N, count)


def test_first_prime_closed_form(orc):
    # the largest prime below 2^60 that is 1 mod 2^11 is 2^60 - 2^14 + 1
    assert orc.ntt_primes(1024, 1)[0] == 2**60 - 2**14 + 1


@pytest.mark.parametrize("N", [2, 16, 1024, 2**16])
def test_psi_and_tables(orc, N):
    q = orc.ntt_primes(N, 1)[0]
    psi = P.pin_psi(orc, q, N)
    if N <= 1024:
        P.pin_tables(orc, q, N, psi)


def test_ntt_roundtrip(orc):
    P.pin_ntt_roundtrip(orc)


def test_polymul_ntt_vs_schoolbook(orc):
    P.pin_polymul_ntt_vs_schoolbook(orc)


def test_polymul_large(orc):
    P.pin_polymul_large(orc)
