"""Plant one mistake at a time in a copy of the C oracle and check that the
pins catch it. The copy is compiled on the CPU into a temporary directory; the
real oracle is not touched."""
import os
import subprocess

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "pm_oracle.c")

# (id, text in the oracle, replacement, pins expected to notice)
MUTANTS = [
    ("wrap_sign", "c[k - N] = or_submod(c[k - N], p, q);", "c[k - N] = or_addmod(c[k - N], p, q);",
     [P.pin_schoolbook_bruteforce, P.pin_closed_forms]),
    ("dropped_term", "c[k] = or_addmod(c[k], p, q);", "{ if (j) c[k] = or_addmod(c[k], p, q); }",
     [P.pin_schoolbook_bruteforce, P.pin_closed_forms]),
    ("coeff_index", "or_mulmod(a[i], b[k + N - i], q)", "or_mulmod(a[i], b[k + N - i - 1], q)",
     [P.pin_coeff]),
    ("fwd_point_index", "uint64_t x = psi_br[h + t];", "uint64_t x = psi_br[h + (t + 1) % h];",
     [P.pin_ntt_eval, P.pin_ntt_invariants]),
    ("fwd_sign", "a[2 * t + 1] = or_submod(tmp[t], xo, q);", "a[2 * t + 1] = or_submod(xo, tmp[t], q);",
     [P.pin_ntt_eval, P.pin_ntt_invariants]),
    ("fwd_even_odd_swapped", "tmp[i] = a[2 * i];\n        tmp[h + i] = a[2 * i + 1];",
     "tmp[i] = a[2 * i + 1];\n        tmp[h + i] = a[2 * i];",
     [P.pin_ntt_eval, P.pin_ntt_invariants]),
    ("fwd_output_pairs", "a[2 * t] = or_addmod(tmp[t], xo, q);", "a[t] = or_addmod(tmp[t], xo, q);",
     [P.pin_ntt_eval]),
    ("inv_transposed", "tmp[h + t] = or_mulmod(or_submod(u, v, q), psi_inv_br[h + t], q);",
     "tmp[h + t] = or_mulmod(or_submod(v, u, q), psi_inv_br[h + t], q);",
     [lambda o: P.pin_ntt_roundtrip(o, sizes=(8, 64)),
      lambda o: P.pin_polymul_ntt_vs_schoolbook(o, sizes=(4, 16))]),
    ("inv_point_forward_table", "tmp[h + t] = or_mulmod(or_submod(u, v, q), psi_inv_br[h + t], q);",
     "tmp[h + t] = or_mulmod(or_submod(u, v, q), psi_inv_br[h + t] == 1 ? 1 : q - psi_inv_br[h + t], q);",
     [lambda o: P.pin_ntt_roundtrip(o, sizes=(8, 64))]),
    ("inv_interleave", "y[2 * i] = tmp[i];\n        y[2 * i + 1] = tmp[h + i];",
     "y[i] = tmp[i];\n        y[h + i] = tmp[h + i];",
     [lambda o: P.pin_ntt_roundtrip(o, sizes=(8, 64))]),
    ("no_inverse_scaling", "for (size_t j = 0; j < N; j++) a[j] = or_mulmod(a[j], ninv, q);", "",
     [lambda o: P.pin_ntt_roundtrip(o, sizes=(8, 64))]),
    ("pointwise_dropped", "c[j] = or_mulmod(c[j], tb[j], q);", "c[j] = or_addmod(c[j], tb[j], q);",
     [lambda o: P.pin_polymul_ntt_vs_schoolbook(o, sizes=(4, 16))]),
    ("bitrev_width", "unsigned bits = ilog2(N);\n    uint64_t psi_inv",
     "unsigned bits = ilog2(N) + 1;\n    uint64_t psi_inv",
     [lambda o: P.pin_tables(o, 12289, 16, 1945), P.pin_ntt_eval]),
    ("eval_point", "uint64_t point = or_powmod(psi, 2 * (uint64_t)bitrev(p, bits) + 1, q);",
     "uint64_t point = or_powmod(psi, 2 * (uint64_t)p + 1, q);",
     [P.pin_ntt_eval]),
    ("mulmod_reduction", "return (uint64_t)(((u128)a * (u128)b) % q);",
     "return (uint64_t)(((u128)a * (u128)b) % q) % (q - 1 ? q - 1 : 1);",
     [P.pin_arith]),
    ("submod_order", "return (uint64_t)(((u128)a + (u128)q - (u128)(b % q)) % q);",
     "return (uint64_t)(((u128)b + (u128)q - (u128)(a % q)) % q);",
     [P.pin_arith]),
    ("prime_skip", "        k--;\n    }\n    return found;", "        k -= 2;\n    }\n    return found;",
     [lambda o: P.pin_ntt_primes(o, 2**14, 8)]),
    ("mr_one_base", "for (int i = 0; i < 12; i++) {\n        uint64_t x = or_powmod(bases[i], d, n);",
     "for (int i = 0; i < 1; i++) {\n        uint64_t x = or_powmod(bases[i], d, n);",
     [P.pin_is_prime]),
    ("psi_not_qnr", "if (or_powmod(g, (q - 1) / 2, q) == q - 1)", "if (or_powmod(g, (q - 1) / 4, q) == q - 1)",
     [lambda o: P.pin_psi(o, o.ntt_primes(16, 1)[0], 16)]),
    ("horner_order", "for (size_t i = N; i-- > 0;) r = or_addmod(or_mulmod(r, x, q), a[i], q);",
     "for (size_t i = 0; i < N; i++) r = or_addmod(or_mulmod(r, x, q), a[i], q);",
     [P.pin_eval]),
]


@pytest.mark.parametrize("mid,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, mid, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must occur exactly once: " + mid
    mut = tmp_path / ("oracle_%s.c" % mid)
    mut.write_text(src.replace(old, new))
    so = tmp_path / ("liboracle_%s.so" % mid)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", str(so), str(mut)])
    o = oracle.Oracle(oracle.load(str(so)))
    caught = 0
    for pin in pins:
        try:
            pin(o)
        except AssertionError:
            caught += 1
    assert caught >= 1, "planted mistake %s passed every pin" % mid
