"""The fused polynomial multiplication of Sec. III-B, in pure Python integers,
for small N, written from what each step computes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): it models the
algorithm, so that its readings can be checked against the plain definition
of the product (``bruteforce.negacyclic``); it shares nothing with the HIP
library.

What the steps compute. Let alpha_i = psi_br[N/2 + i] = psi^(2 br_{n-1}(i) + 1)
for i < N/2: the full forward transform holds a(alpha_i) and a(-alpha_i) at
positions 2i and 2i+1 (R2 reading), and x^N + 1 is the product of the N/2
quadratics x^2 - alpha_i^2.

  ct_truncated          the forward transform without its last stage (stride
                        1): at positions 2i, 2i+1 the residue v0 + v1 x of a
                        modulo x^2 - alpha_i^2 (the last stage would map it to
                        v0 +- alpha_i v1 = a(+-alpha_i)); computed here from
                        the residue's definition, v0 = a_even(alpha_i^2),
                        v1 = a_odd(alpha_i^2).
  gs_truncated          the halved inverse without one stage. reading="first"
                        omits the first stage (stride 1, which with its 1/2
                        maps the two values back to the residue pair): the
                        rest interpolates c from its residue pairs, so it is
                        computed as the inverse transform (definition: 1/N
                        times the sum over the points) of the values
                        v0 +- alpha_i v1. reading="last" is the text's literal
                        loop change, which keeps the first stage and omits
                        the last one (stride N/2, twiddle psi^-N/2, halved):
                        its output is that last stage undone on the full
                        inverse, z_j = c_j + psi^(N/2) c_(j+N/2),
                        z_(j+N/2) = c_j - psi^(N/2) c_(j+N/2).
  fused_pair            Alg. 7: the product of two residues modulo
                        x^2 - gamma, (a0 + a1 x)(b0 + b1 x) =
                        (a0 b0 + gamma a1 b1) + (a0 b1 + a1 b0) x, with the
                        cross term from one product of sums (Karatsuba): four
                        modular products instead of five.
  fused_pair_reference  what the fused pair replaces, by definition: the last
                        CT butterflies of a and b with alpha, the pointwise
                        product, the first GS butterfly with alpha^-1, halved.
  polymul_fused         Alg. 8: truncated transforms of a and b, Alg. 7 on
                        each pair with gamma_i = alpha_i^2 taken as
                        (-1)^i psi_br[N/4 + floor(i/2)] (reading R7b), then
                        the truncated inverse.
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


def _poly_at(coeffs, x, q):
    return sum(c * pow(x, j, q) for j, c in enumerate(coeffs)) % q


def ct_truncated(a, q, psi_br):
    n = len(a)
    a = [int(v) % q for v in a]
    out = [0] * n
    for i in range(n // 2):
        gamma = psi_br[n // 2 + i] ** 2 % q
        out[2 * i] = _poly_at(a[0::2], gamma, q)
        out[2 * i + 1] = _poly_at(a[1::2], gamma, q)
    return out


def _inverse_transform(y, q, psi_br):
    """c_j = (1/N) sum_p y_p x_p^-j over the points x_p = psi^(2 br(p) + 1),
    i.e. +-alpha_i at positions 2i, 2i+1."""
    n = len(y)
    points = []
    for i in range(n // 2):
        alpha = psi_br[n // 2 + i]
        points += [alpha, (q - alpha) % q]
    n_inv = pow(n, q - 2, q)
    inv_points = [pow(x, q - 2, q) for x in points]
    return [n_inv * sum(yp * pow(xi, j, q) for yp, xi in zip(y, inv_points)) % q for j in range(n)]


def gs_truncated(w, q, psi_br, reading="first"):
    n = len(w)
    w = [int(v) % q for v in w]
    values = []
    for i in range(n // 2):
        alpha = psi_br[n // 2 + i]
        values += [(w[2 * i] + alpha * w[2 * i + 1]) % q, (w[2 * i] - alpha * w[2 * i + 1]) % q]
    if reading == "first":
        return _inverse_transform(values, q, psi_br)
    if reading == "last":
        c = _inverse_transform(w, q, psi_br)          # the pairs taken as transform values
        s = psi_br[1]                                  # psi^(N/2), the inverse of the stage's twiddle
        h = n // 2
        return [(c[j] + s * c[j + h]) % q for j in range(h)] + [(c[j] - s * c[j + h]) % q for j in range(h)]
    raise ValueError(reading)


def fused_pair(a0, a1, b0, b1, gamma, q):
    lo = a0 * b0 % q
    hi = a1 * b1 % q
    cross = ((a0 + a1) * (b0 + b1) - lo - hi) % q
    return (lo + gamma * hi) % q, cross


def fused_pair_reference(a0, a1, b0, b1, alpha, q):
    half = (q + 1) // 2
    ua, va = (a0 + alpha * a1) % q, (a0 - alpha * a1) % q
    ub, vb = (b0 + alpha * b1) % q, (b0 - alpha * b1) % q
    u, v = ua * ub % q, va * vb % q
    alpha_inv = pow(alpha, q - 2, q)
    return (u + v) * half % q, alpha_inv * (u - v) % q * half % q


def polymul_fused(a, b, q, psi_br, psi_inv_br, reading="first"):
    """psi_inv_br is accepted for the interface of the device entry point; the
    inverse here is computed from its definition with the points of psi_br."""
    n = len(a)
    A = ct_truncated(a, q, psi_br)
    B = ct_truncated(b, q, psi_br)
    C = [0] * n
    for i in range(n // 2):
        g = psi_br[n // 4 + i // 2]
        gamma = g if i % 2 == 0 else (q - g) % q
        C[2 * i], C[2 * i + 1] = fused_pair(A[2 * i], A[2 * i + 1], B[2 * i], B[2 * i + 1], gamma, q)
    return gs_truncated(C, q, psi_br, reading)
