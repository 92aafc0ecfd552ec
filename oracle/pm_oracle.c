/*
 * Oracle for exact negacyclic polynomial multiplication in Z_q[x]/(x^N + 1).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * CPU reference that the GPU library is checked against. Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it. It
 * shares no code, header, table or constant with the GPU library, and the
 * GPU library never calls it.
 *
 * Every reduction here is the textbook one, x mod q = x - floor(x/q)*q
 * (Sec. II-A), done with the C '%' operator on unsigned __int128. There is no
 * Barrett reduction, no halving trick and no blocking or reordering.
 *
 * Functions and the passages they follow:
 *   or_mulmod / or_mulmod_vec / or_addmod / or_submod / or_powmod
 *       modular arithmetic of Z_q (Sec. III, opening definition of Z_m).
 *   or_polymul_schoolbook / or_polymul_coeff
 *       the negacyclic convolution, i.e. the product in Z_q[x]/(x^N + 1)
 *       (Sec. III): c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j.
 *   or_ntt_fwd
 *       the forward transform Alg. 5 computes (Sec. III-A), normal order in,
 *       bit-reversed order out, written from its definition: the values of
 *       the polynomial at the roots psi^(2 br(p) + 1) of x^N = -1, computed
 *       by the recursive even/odd split a(x) = a_e(x^2) + x a_o(x^2) (a
 *       decimation-in-time recursion, not Alg. 5's butterfly loops); the
 *       points are read from the table psi_br[i] = psi^br(i).
 *   or_ntt_inv
 *       its inverse (what Alg. 6 with the 1/N of Eq. 1 computes): the same
 *       recursion undone level by level with psi^-1 points, without the
 *       factors 1/2, followed by an explicit multiplication by
 *       N^-1 = N^(q-2) mod q; it does not use the per-butterfly halving of
 *       Eq. 2.
 *   or_ntt_eval
 *       brute-force definition of the forward transform: output position p
 *       is a(psi^(2*br(p)+1)) (evaluation at the odd powers of psi, in
 *       bit-reversed order; the reading under Alg. 5 of "bit-reversed order").
 *   or_polymul_ntt
 *       Eq. 1: c = (1/N) GS_{psi^-1}(CT_psi(a) . CT_psi(b)).
 *   or_poly_eval
 *       Horner evaluation of a polynomial at one point of Z_q.
 *   or_is_prime / or_ntt_primes / or_find_psi / or_psi_tables
 *       parameter generation: primes q = 1 mod 2N below 2^bits in
 *       descending order, a primitive 2N-th root of unity psi (setup of
 *       Sec. III-A: q prime, 2N | q-1, psi of order 2N), and the bit-reversed
 *       twiddle tables of Alg. 5/6.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * (u128)b) % q);
}

/* c[i] = a[i]*b[i] mod q for i < n (elementwise definition of the product). */
void or_mulmod_vec(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t n, uint64_t q) {
    for (size_t i = 0; i < n; i++) c[i] = or_mulmod(a[i], b[i], q);
}

uint64_t or_addmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + (u128)b) % q);
}

uint64_t or_submod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + (u128)q - (u128)(b % q)) % q);
}

uint64_t or_powmod(uint64_t base, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    base %= q;
    while (e) {
        if (e & 1) r = or_mulmod(r, base, q);
        base = or_mulmod(base, base, q);
        e >>= 1;
    }
    return r;
}

/* Reverse the low `bits` bits of i. */
static size_t bitrev(size_t i, unsigned bits) {
    size_t r = 0;
    for (unsigned b = 0; b < bits; b++) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

static unsigned ilog2(size_t n) {
    unsigned l = 0;
    while (((size_t)1 << l) < n) l++;
    return l;
}

/* ---------------------------------------------------------------------- */
/* Negacyclic convolution, straight from its definition.                   */
/* ---------------------------------------------------------------------- */

void or_polymul_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *c,
                           size_t N, uint64_t q) {
    for (size_t k = 0; k < N; k++) c[k] = 0;
    for (size_t i = 0; i < N; i++) {
        for (size_t j = 0; j < N; j++) {
            uint64_t p = or_mulmod(a[i], b[j], q);
            size_t k = i + j;
            if (k < N)
                c[k] = or_addmod(c[k], p, q);       /* x^k term */
            else
                c[k - N] = or_submod(c[k - N], p, q); /* x^N = -1 */
        }
    }
}

/* One coefficient c_k of the negacyclic product, O(N). */
uint64_t or_polymul_coeff(const uint64_t *a, const uint64_t *b, size_t N,
                          uint64_t q, size_t k) {
    uint64_t pos = 0, neg = 0;
    for (size_t i = 0; i <= k; i++) pos = or_addmod(pos, or_mulmod(a[i], b[k - i], q), q);
    for (size_t i = k + 1; i < N; i++) neg = or_addmod(neg, or_mulmod(a[i], b[k + N - i], q), q);
    return or_submod(pos, neg, q);
}

/* Horner evaluation a(x) mod q. */
uint64_t or_poly_eval(const uint64_t *a, size_t N, uint64_t q, uint64_t x) {
    uint64_t r = 0;
    for (size_t i = N; i-- > 0;) r = or_addmod(or_mulmod(r, x, q), a[i], q);
    return r;
}

/* ---------------------------------------------------------------------- */
/* The transforms, from their definition as evaluation and interpolation.  */
/* ---------------------------------------------------------------------- */

/*
 * Forward transform (what Alg. 5 computes, Sec. III-A): out[p] = a(x_p) with
 * x_p = psi^(2 br(p) + 1), the N roots of x^N = -1 taken in bit-reversed
 * order. Computed by the even/odd split of the polynomial,
 *     a(x) = a_even(x^2) + x * a_odd(x^2),
 * not by the butterfly loops of Alg. 5:
 *   - positions 2t and 2t+1 hold the points x and -x for
 *     x = psi^(2 br_{n-1}(t) + 1), since br_n(2t+1) = br_n(2t) + N/2 and
 *     psi^N = -1;
 *   - x^2 = (psi^2)^(2 br_{n-1}(t) + 1) is point t of the same transform of
 *     size N/2 with psi^2 (whose (N/2)-th power is again -1);
 * so out[2t] = E[t] + x O[t] and out[2t+1] = E[t] - x O[t], where E and O are
 * the size-N/2 transforms of the even and odd coefficients. At a level of
 * size M (root psi^(N/M)) the point x for position pair t is the table entry
 * psi_br[M/2 + t] = psi^br_n(M/2 + t) = psi^((N/M) (2 br_{m-1}(t) + 1)).
 *
 * a: M coefficients, replaced by the M values; tmp: M words of scratch.
 */
static void eval_even_odd(uint64_t *a, size_t M, uint64_t q, const uint64_t *psi_br, uint64_t *tmp) {
    if (M == 1) return;                     /* a constant is its own value */
    size_t h = M / 2;
    for (size_t i = 0; i < h; i++) {        /* even coefficients, then odd ones */
        tmp[i] = a[2 * i];
        tmp[h + i] = a[2 * i + 1];
    }
    eval_even_odd(tmp, h, q, psi_br, a);        /* E, with a as scratch */
    eval_even_odd(tmp + h, h, q, psi_br, a);    /* O */
    for (size_t t = 0; t < h; t++) {
        uint64_t x = psi_br[h + t];
        uint64_t xo = or_mulmod(x, tmp[h + t], q);
        a[2 * t] = or_addmod(tmp[t], xo, q);
        a[2 * t + 1] = or_submod(tmp[t], xo, q);
    }
}

/*
 * The inverse of eval_even_odd up to a factor M: from the values y at the
 * points of a size-M level, E[t] = (y[2t] + y[2t+1]) / 2 and
 * O[t] = (y[2t] - y[2t+1]) / (2x); the factors 1/2 are left out here, so each
 * level doubles and the result is M times the coefficients. The inverse
 * point 1/x is psi_inv_br[M/2 + t] (the table of psi^-1).
 */
static void interp_even_odd(uint64_t *y, size_t M, uint64_t q, const uint64_t *psi_inv_br, uint64_t *tmp) {
    if (M == 1) return;
    size_t h = M / 2;
    for (size_t t = 0; t < h; t++) {
        uint64_t u = y[2 * t], v = y[2 * t + 1];
        tmp[t] = or_addmod(u, v, q);                                   /* 2 E[t] */
        tmp[h + t] = or_mulmod(or_submod(u, v, q), psi_inv_br[h + t], q);  /* 2 O[t] */
    }
    interp_even_odd(tmp, h, q, psi_inv_br, y);      /* M * even coefficients */
    interp_even_odd(tmp + h, h, q, psi_inv_br, y);  /* M * odd coefficients */
    for (size_t i = 0; i < h; i++) {
        y[2 * i] = tmp[i];
        y[2 * i + 1] = tmp[h + i];
    }
}

void or_ntt_fwd(uint64_t *a, size_t N, uint64_t q, const uint64_t *psi_br) {
    uint64_t *tmp = (uint64_t *)malloc(N * sizeof(uint64_t));
    eval_even_odd(a, N, q, psi_br, tmp);
    free(tmp);
}

void or_ntt_inv(uint64_t *a, size_t N, uint64_t q, const uint64_t *psi_inv_br) {
    uint64_t *tmp = (uint64_t *)malloc(N * sizeof(uint64_t));
    interp_even_odd(a, N, q, psi_inv_br, tmp);
    free(tmp);
    /* the 1/N factor of Eq. 1, as an explicit multiplication */
    uint64_t ninv = or_powmod(N % q, q - 2, q);
    for (size_t j = 0; j < N; j++) a[j] = or_mulmod(a[j], ninv, q);
}

/* Brute-force forward transform: out[p] = a(psi^(2 br(p) + 1)). O(N^2). */
void or_ntt_eval(const uint64_t *a, uint64_t *out, size_t N, uint64_t q, uint64_t psi) {
    unsigned bits = ilog2(N);
    for (size_t p = 0; p < N; p++) {
        uint64_t point = or_powmod(psi, 2 * (uint64_t)bitrev(p, bits) + 1, q);
        out[p] = or_poly_eval(a, N, q, point);
    }
}

/* Eq. 1 on one pair of polynomials; a, b are left untouched. */
void or_polymul_ntt(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t N,
                    uint64_t q, const uint64_t *psi_br, const uint64_t *psi_inv_br) {
    uint64_t *tb = (uint64_t *)malloc(N * sizeof(uint64_t));
    memcpy(c, a, N * sizeof(uint64_t));
    memcpy(tb, b, N * sizeof(uint64_t));
    or_ntt_fwd(c, N, q, psi_br);
    or_ntt_fwd(tb, N, q, psi_br);
    for (size_t j = 0; j < N; j++) c[j] = or_mulmod(c[j], tb[j], q);
    or_ntt_inv(c, N, q, psi_inv_br);
    free(tb);
}

/* ---------------------------------------------------------------------- */
/* Parameters: primes, psi, twiddle tables.                                */
/* ---------------------------------------------------------------------- */

/* Deterministic Miller-Rabin; the first 12 prime bases are exact for
 * every n < 3.3e24, hence for every 64-bit n. */
int or_is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    uint64_t d = n - 1;
    unsigned s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = or_powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (unsigned r = 1; r < s; r++) {
            x = or_mulmod(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* The `count` largest primes q < 2^bits with q = 1 (mod two_n), in
 * descending order. Returns how many were found. */
size_t or_ntt_primes(uint64_t two_n, unsigned bits, size_t count, uint64_t *out) {
    size_t found = 0;
    uint64_t top = (bits >= 64) ? UINT64_MAX : (((uint64_t)1 << bits) - 1);
    uint64_t k = (top - 1) / two_n;          /* largest k with k*2N + 1 <= top */
    while (found < count && k >= 1) {
        uint64_t q = k * two_n + 1;
        if (or_is_prime(q)) out[found++] = q;
        k--;
    }
    return found;
}

/* psi = g^((q-1)/(2N)) for the smallest quadratic non-residue g >= 2,
 * i.e. g^((q-1)/2) = -1. Then psi^N = -1 and psi has order exactly 2N.
 * Returns 0 if q is not 1 mod 2N. */
uint64_t or_find_psi(uint64_t q, size_t N) {
    if ((q - 1) % (2 * (uint64_t)N) != 0) return 0;
    for (uint64_t g = 2; g < q; g++) {
        if (or_powmod(g, (q - 1) / 2, q) == q - 1)
            return or_powmod(g, (q - 1) / (2 * (uint64_t)N), q);
    }
    return 0;
}

/* psi_br[i] = psi^br(i), psi_inv_br[i] = psi^-br(i), br over log2(N) bits. */
void or_psi_tables(uint64_t q, size_t N, uint64_t psi, uint64_t *psi_br, uint64_t *psi_inv_br) {
    unsigned bits = ilog2(N);
    uint64_t psi_inv = or_powmod(psi, 2 * (uint64_t)N - 1, q);   /* psi^(2N) = 1 */
    for (size_t i = 0; i < N; i++) {
        uint64_t e = bitrev(i, bits);
        psi_br[i] = or_powmod(psi, e, q);
        psi_inv_br[i] = or_powmod(psi_inv, e, q);
    }
}
