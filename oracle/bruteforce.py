"""Pure-Python big-integer brute force for tiny inputs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Independent of ``pm_oracle.c``: nothing here calls the C library. It gives a
second, differently written route to the same definitions, used to pin the C
oracle on tiny sizes (N <= 64 or so):

  negacyclic(a, b, q)      product in Z_q[x]/(x^N+1) by expanding a(x)b(x) in
                           Z[x] and folding x^(N+t) = -x^t (Sec. III).
  eval_poly(a, x, q)       a(x) mod q, term by term.
  ntt_by_evaluation        output p = a(psi^(2 br(p) + 1)).
  is_prime_mr(n)           Miller-Rabin with a different base set than the C
                           oracle (the first 13 primes, run as a separate loop).
  is_prime_trial(n)        trial division, for small n.
"""
from __future__ import annotations


def bitrev(i: int, bits: int) -> int:
    return int(format(i, "0%db" % bits)[::-1], 2) if bits else 0


def negacyclic(a, b, q):
    n = len(a)
    full = [0] * (2 * n)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            full[i + j] += int(ai) * int(bj)
    return [(full[t] - full[t + n]) % q for t in range(n)]


def eval_poly(a, x, q):
    return sum(int(ai) * pow(x, i, q) for i, ai in enumerate(a)) % q


def ntt_by_evaluation(a, q, psi):
    n = len(a)
    bits = n.bit_length() - 1
    return [eval_poly(a, pow(psi, 2 * bitrev(p, bits) + 1, q), q) for p in range(n)]


def is_prime_trial(n: int) -> bool:
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def is_prime_mr(n: int) -> bool:
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True
