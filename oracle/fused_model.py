"""The fused polynomial multiplication of Sec. III-B, step by step, in pure
Python integers, for small N.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): it models the
algorithm, so that its readings can be checked against the plain definition
of the product (``bruteforce.negacyclic``); it shares nothing with the HIP
library.

  ct_merged_truncated   Alg. 5 with the final stage omitted (the loop runs
                        while m < N/2).
  gs_merged_truncated   Alg. 6 without one stage, each butterfly output
                        halved (Eq. 2's merged 1/N). reading="first" omits
                        the first stage (m = N/2), which is what the fused
                        product needs; reading="last" is the text's literal
                        loop change (while m > 1), which omits m = 1.
  fused_pair            Alg. 7: (a0, a1), (b0, b1), alpha^2 ->
                        (a0 b0 + alpha^2 a1 b1, a0 b1 + a1 b0) with four
                        products (Karatsuba).
  fused_pair_reference  the same pair by its definition: the last CT
                        butterflies of a and b with alpha, the product, the
                        first GS butterfly with alpha^-1, times 1/2.
  polymul_fused         Alg. 8.
"""
from __future__ import annotations


def bitrev(i: int, bits: int) -> int:
    return int(format(i, "0%db" % bits)[::-1], 2) if bits else 0


def tables(q: int, n: int, psi: int):
    """psi_br[i] = psi^br(i), psi_inv_br[i] = psi^-br(i) (Sec. III-A)."""
    bits = n.bit_length() - 1
    inv = pow(psi, 2 * n - 1, q)
    return ([pow(psi, bitrev(i, bits), q) for i in range(n)],
            [pow(inv, bitrev(i, bits), q) for i in range(n)])


def ct_merged_truncated(a, q, psi_br):
    x = [int(v) % q for v in a]
    n = len(x)
    m, k = 1, n // 2
    while m < n // 2:
        for i in range(m):
            xi = psi_br[m + i]
            for j in range(2 * i * k, 2 * i * k + k):
                t = xi * x[j + k] % q
                x[j], x[j + k] = (x[j] + t) % q, (x[j] - t) % q
        m, k = 2 * m, k // 2
    return x


def gs_merged_truncated(x, q, psi_inv_br, reading="first"):
    x = [int(v) % q for v in x]
    n = len(x)
    half = (q + 1) // 2
    if reading == "first":
        m, k, stop = n // 4, 2, 1          # stages m = N/4 .. 1
    elif reading == "last":
        m, k, stop = n // 2, 1, 2          # stages m = N/2 .. 2
    else:
        raise ValueError(reading)
    while m >= stop:
        for i in range(m):
            xi = psi_inv_br[m + i]
            for j in range(2 * i * k, 2 * i * k + k):
                u, v = x[j], x[j + k]
                x[j] = (u + v) * half % q
                x[j + k] = xi * ((u - v) * half % q) % q
        m, k = m // 2, 2 * k
    return x


def fused_pair(a0, a1, b0, b1, alpha2, q):
    prod1 = a0 * b0 % q
    prod2 = a1 * b1 % q
    sum1 = (a0 + a1) % q
    sum2 = (b0 + b1) % q
    prod3 = sum1 * sum2 % q
    prod4 = alpha2 * prod2 % q
    return (prod1 + prod4) % q, ((prod3 - prod1) % q - prod2) % q


def fused_pair_reference(a0, a1, b0, b1, alpha, q):
    half = (q + 1) // 2
    ua, va = (a0 + alpha * a1) % q, (a0 - alpha * a1) % q
    ub, vb = (b0 + alpha * b1) % q, (b0 - alpha * b1) % q
    u, v = ua * ub % q, va * vb % q
    alpha_inv = pow(alpha, q - 2, q)
    return (u + v) * half % q, alpha_inv * (u - v) % q * half % q


def polymul_fused(a, b, q, psi_br, psi_inv_br, reading="first"):
    n = len(a)
    A = ct_merged_truncated(a, q, psi_br)
    B = ct_merged_truncated(b, q, psi_br)
    C = [0] * n
    for i in range(n // 2):
        u = A[2 * i] * B[2 * i] % q
        v = A[2 * i + 1] * B[2 * i + 1] % q
        w = (A[2 * i] + A[2 * i + 1]) * (B[2 * i] + B[2 * i + 1]) % q
        y = (w - u) % q
        C[2 * i + 1] = (y - v) % q
        z = v * psi_br[n // 4 + i // 2] % q
        C[2 * i] = (u + z) % q if i % 2 == 0 else (u - z) % q
    return gs_merged_truncated(C, q, psi_inv_br, reading)
