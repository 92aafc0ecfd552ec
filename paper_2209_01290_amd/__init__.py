"""Exact negacyclic polynomial multiplication in Z_q[x]/(x^N + 1) on MI355X.

The product is computed as in Eq. 2 of the paper: a merged Cooley-Tukey
forward NTT (normal order in, bit-reversed out, psi powers folded into the
twiddles, Alg. 5), a pointwise product mod q, and a merged Gentleman-Sande
inverse NTT (bit-reversed in, normal out, Alg. 6) whose butterflies halve both
outputs, which merges the 1/N scaling. Words are 64 bits wide, q < 2^62, and
every product is reduced by the paper's Barrett variant (Alg. 4).

Submodules:
  lib     ctypes binding of the C-ABI library ``libpm.so`` (HIP kernels for gfx950)
  build   compiles the library with hipcc
  synth   seeded synthetic inputs (SplitMix64), shared by tests and benchmarks
  serve   continuous-batching request loop over the batched entry points

Importing this package loads nothing; ``lib`` loads the shared library on
first use and raises if it is missing.
"""
__all__ = ["lib", "build", "synth", "serve"]
