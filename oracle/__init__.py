"""CPU oracle for exact negacyclic polynomial multiplication.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers. The GPU library never imports this
package, and this package never imports the GPU library.

This module is a thin ctypes binding over ``pm_oracle.c`` (plain C, every
reduction by ``%`` on ``unsigned __int128``). It compiles that file with gcc on
first use when the shared object is missing. Arrays are numpy ``uint64``.

Parity status of every function is pinned by tests under ``tests/`` that
check it against mathematics the paper fixes (closed forms, brute force on tiny
inputs, invariants of the transform); see the module docstrings there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc -O2 into a shared object; returns its path."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _declare(lib):
    u64, sz = ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "or_mulmod": (u64, [u64, u64, u64]),
        "or_mulmod_vec": (None, [_u64p, _u64p, _u64p, sz, u64]),
        "or_addmod": (u64, [u64, u64, u64]),
        "or_submod": (u64, [u64, u64, u64]),
        "or_powmod": (u64, [u64, u64, u64]),
        "or_polymul_schoolbook": (None, [_u64p, _u64p, _u64p, sz, u64]),
        "or_polymul_coeff": (u64, [_u64p, _u64p, sz, u64, sz]),
        "or_poly_eval": (u64, [_u64p, sz, u64, u64]),
        "or_ntt_fwd": (None, [_u64p, sz, u64, _u64p]),
        "or_ntt_inv": (None, [_u64p, sz, u64, _u64p]),
        "or_ntt_eval": (None, [_u64p, _u64p, sz, u64, u64]),
        "or_polymul_ntt": (None, [_u64p, _u64p, _u64p, sz, u64, _u64p, _u64p]),
        "or_is_prime": (ctypes.c_int, [u64]),
        "or_ntt_primes": (sz, [u64, ctypes.c_uint, sz, _u64p]),
        "or_find_psi": (u64, [u64, sz]),
        "or_psi_tables": (None, [u64, sz, u64, _u64p, _u64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def load(path: str | None = None):
    """Load (building if needed) the oracle library. ``path`` loads a variant."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            _lib = _declare(ctypes.CDLL(build()))
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], "need contiguous uint64"
    return a.ctypes.data_as(_u64p)


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.uint64)


class Oracle:
    """Object form, so a test can run the same pins against a planted variant."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # -- arithmetic of Z_q -------------------------------------------------
    def mulmod(self, a, b, q):
        return int(self.lib.or_mulmod(a, b, q))

    def addmod(self, a, b, q):
        return int(self.lib.or_addmod(a, b, q))

    def submod(self, a, b, q):
        return int(self.lib.or_submod(a, b, q))

    def powmod(self, a, e, q):
        return int(self.lib.or_powmod(a, e, q))

    def mulmod_vec(self, a, b, q):
        """Elementwise a*b mod q (the pm_barrett_mulmod definition)."""
        a, b = _u64(a), _u64(b)
        c = np.empty_like(a)
        self.lib.or_mulmod_vec(_p(a), _p(b), _p(c), a.size, q)
        return c

    # -- polynomials -------------------------------------------------------
    def polymul_schoolbook(self, a, b, q):
        a, b = _u64(a), _u64(b)
        c = np.empty_like(a)
        self.lib.or_polymul_schoolbook(_p(a), _p(b), _p(c), a.size, q)
        return c

    def polymul_coeff(self, a, b, q, k):
        a, b = _u64(a), _u64(b)
        return int(self.lib.or_polymul_coeff(_p(a), _p(b), a.size, q, k))

    def poly_eval(self, a, q, x):
        a = _u64(a)
        return int(self.lib.or_poly_eval(_p(a), a.size, q, x))

    def ntt_fwd(self, a, q, psi_br):
        x = _u64(a).copy()
        self.lib.or_ntt_fwd(_p(x), x.size, q, _p(_u64(psi_br)))
        return x

    def ntt_inv(self, a, q, psi_inv_br):
        x = _u64(a).copy()
        self.lib.or_ntt_inv(_p(x), x.size, q, _p(_u64(psi_inv_br)))
        return x

    def ntt_eval(self, a, q, psi):
        a = _u64(a)
        out = np.empty_like(a)
        self.lib.or_ntt_eval(_p(a), _p(out), a.size, q, psi)
        return out

    def polymul_ntt(self, a, b, q, psi_br, psi_inv_br):
        a, b = _u64(a), _u64(b)
        c = np.empty_like(a)
        self.lib.or_polymul_ntt(_p(a), _p(b), _p(c), a.size, q,
                                _p(_u64(psi_br)), _p(_u64(psi_inv_br)))
        return c

    # -- parameters --------------------------------------------------------
    def is_prime(self, n):
        return bool(self.lib.or_is_prime(n))

    def ntt_primes(self, N, count, bits=60):
        out = np.zeros(count, dtype=np.uint64)
        got = self.lib.or_ntt_primes(2 * N, bits, count, _p(out))
        return [int(x) for x in out[:got]]

    def find_psi(self, q, N):
        return int(self.lib.or_find_psi(q, N))

    def psi_tables(self, q, N, psi=None):
        if psi is None:
            psi = self.find_psi(q, N)
        fwd = np.empty(N, dtype=np.uint64)
        inv = np.empty(N, dtype=np.uint64)
        self.lib.or_psi_tables(q, N, psi, _p(fwd), _p(inv))
        return fwd, inv


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def __getattr__(name):  # module-level convenience: oracle.polymul_ntt(...)
    if name.startswith("_"):
        raise AttributeError(name)
    return getattr(default(), name)
