"""Seeded synthetic inputs: uniform coefficients in [0, q).

This module holds no arithmetic of the method. It only draws random words, so
both the GPU path and the CPU oracle can be fed the very same operands.

Generator: SplitMix64's output function (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used in counter mode:

    mix(z)    = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
                z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
    key(seed, ids...) : k = mix(seed); for each id: k = mix(k + G*(id+1))
    word(k, j) = mix(k + G*(j+1)),        G = 0x9E3779B97F4A7C15

A coefficient takes the top len(q) bits of its word and is redrawn from the
same counter under the key mix(k ^ attempt) while it is >= q, so every value is
uniform on [0, q). All arithmetic is modulo 2^64.

Stream ids name an operand: (request, limb, poly, operand) with operand 0 for a
and 1 for b. Seeds are 220901290 + k for workload k (the paper's arXiv id).
"""
from __future__ import annotations

import numpy as np

G = np.uint64(0x9E3779B97F4A7C15)
C1 = np.uint64(0xBF58476D1CE4E5B9)
C2 = np.uint64(0x94D049BB133111EB)
SEED_BASE = 220901290

_M64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.array(z, dtype=np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= C1
        z ^= z >> np.uint64(27)
        z *= C2
        z ^= z >> np.uint64(31)
    return z


def _mix_int(z: int) -> int:
    z &= _M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def key(seed: int, *ids: int) -> int:
    k = _mix_int(seed)
    for i in ids:
        k = _mix_int(k + 0x9E3779B97F4A7C15 * (int(i) + 1))
    return k


def words(k: int, n: int) -> np.ndarray:
    """n raw 64-bit words of stream k."""
    j = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(np.uint64(k) + G * j)


def uniform_mod(k: int, n: int, q: int) -> np.ndarray:
    """n coefficients uniform on [0, q) from stream k."""
    bits = int(q).bit_length()
    shift = np.uint64(64 - bits)
    qq = np.uint64(q)
    with np.errstate(over="ignore"):
        v = words(k, n) >> shift
        bad = np.nonzero(v >= qq)[0]
        attempt = 1
        while bad.size:
            k2 = _mix_int(k ^ attempt)
            j = bad.astype(np.uint64) + np.uint64(1)
            v[bad] = _mix(np.uint64(k2) + G * j) >> shift
            bad = bad[v[bad] >= qq]
            attempt += 1
    return v


def operands(seed: int, q_per_limb, polys: int, N: int, request: int = 0):
    """(a, b) as uint64 arrays of shape [limbs][polys][N]; limb l uses q_per_limb[l]."""
    L = len(q_per_limb)
    a = np.empty((L, polys, N), dtype=np.uint64)
    b = np.empty((L, polys, N), dtype=np.uint64)
    for l, q in enumerate(q_per_limb):
        for p in range(polys):
            a[l, p] = uniform_mod(key(seed, request, l, p, 0), N, int(q))
            b[l, p] = uniform_mod(key(seed, request, l, p, 1), N, int(q))
    return a, b


# ------------------------------------------------------------ on the device --
# The same generator on a HIP device with torch int64 tensors (two's-complement
# wrap-around; logical right shifts are arithmetic shifts masked to the low
# 64-k bits), for workloads too large to draw on the host. Bit-identical to
# uniform_mod (tested).

def _s64(x: int) -> int:
    x &= _M64
    return x - (1 << 64) if x >> 63 else x


def _lsr(z, k):
    import torch
    if isinstance(k, int):
        return torch.bitwise_and(torch.bitwise_right_shift(z, k), (1 << (64 - k)) - 1)
    mask = torch.bitwise_left_shift(torch.ones_like(k), 64 - k) - 1   # k >= 2 here
    return torch.bitwise_and(torch.bitwise_right_shift(z, k), mask)


def _mix_t(z):
    z = z ^ _lsr(z, 30)
    z = z * _s64(0xBF58476D1CE4E5B9)
    z = z ^ _lsr(z, 27)
    z = z * _s64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def uniform_mod_device(keys, n, qs, out):
    """out[s, :n] = uniform_mod(keys[s], n, qs[s]) for every stream s, drawn on
    out's device. out: int64 tensor [S, n]."""
    import torch
    dev = out.device
    S = len(keys)
    assert out.shape[0] == S and out.shape[1] == n
    j = torch.arange(1, n + 1, dtype=torch.int64, device=dev).unsqueeze(0)
    g = _s64(0x9E3779B97F4A7C15)
    kt = torch.tensor([_s64(k) for k in keys], dtype=torch.int64, device=dev).unsqueeze(1)
    qt = torch.tensor([int(q) for q in qs], dtype=torch.int64, device=dev).unsqueeze(1)
    sh = torch.tensor([64 - int(q).bit_length() for q in qs], dtype=torch.int64, device=dev).unsqueeze(1)
    v = _lsr(_mix_t(kt + g * j), sh)
    attempt = 1
    bad = v >= qt
    while bool(bad.any()):
        k2 = torch.tensor([_s64(_mix_int(int(k) ^ attempt)) for k in keys], dtype=torch.int64,
                          device=dev).unsqueeze(1)
        v2 = _lsr(_mix_t(k2 + g * j), sh)
        v = torch.where(bad, v2, v)
        bad = bad & (v2 >= qt)
        attempt += 1
    out.copy_(v)
    return out
