"""The Barrett variant study kernels (Alg. 2, 3, 4 and '%', 32- and 64-bit
words): exact remainders against the oracle and correction counts equal to
the step-by-step models on the very same inputs."""
import numpy as np
import pytest

import oracle
from oracle import barrett_models as B
from paper_2209_01290_amd import synth

pytestmark = pytest.mark.gpu

MODELS = {2: B.classical, 3: B.dhem_palisade, 4: B.proposed}


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


def _run(L, variant, word_bits, q, a, b):
    import torch
    n = a.size
    da, db = L.to_device(a), L.to_device(b)
    dc = torch.empty_like(da)
    hist = torch.zeros(3 * ((n + 255) // 256), dtype=torch.int32, device="cuda")
    L.pm_reduce_apply(variant, word_bits, da, db, dc, hist, q)
    torch.cuda.synchronize()
    return L.to_host(dc), hist.cpu().numpy().reshape(-1, 3).sum(axis=0)


CASES = [(32, 28), (32, 29), (32, 30), (64, 30), (64, 60), (64, 61), (64, 62), (64, 35)]


@pytest.mark.parametrize("word_bits,qbits", CASES)
def test_variants_exact_and_counts(L, word_bits, qbits):
    q = L.pm_ntt_primes(1024, 1, qbits)[0]
    n = 1 << 14
    a = synth.uniform_mod(synth.key(21, qbits, 0), n, q)
    b = synth.uniform_mod(synth.key(21, qbits, 1), n, q)
    a[:4] = [q - 1, q - 1, 0, 1]
    b[:4] = [q - 1, 1, q - 1, q - 1]
    want = oracle.default().mulmod_vec(a, b, q)
    for variant in (0, 2, 3, 4):
        if variant == 3 and qbits > word_bits - 4:
            continue
        got, hist = _run(L, variant, word_bits, q, a, b)
        assert np.array_equal(got, want), (variant, word_bits, qbits)
        assert int(hist.sum()) == n
        if variant == 0:
            continue
        model = MODELS[variant]
        counts = np.zeros(3, np.int64)
        for x, y in zip(a.tolist(), b.tolist()):
            counts[model(x * y, q, beta=word_bits)[1]] += 1
        assert hist.tolist() == counts.tolist(), (variant, word_bits, qbits, hist, counts)
        if variant != 2:
            assert hist[2] == 0


def test_worked_example_corrections(L):
    a, b, q = 994674970, 994705408, 994705409
    A, Bv = np.array([a], np.uint64), np.array([b], np.uint64)
    for variant, k in [(2, 2), (4, 1)]:
        got, hist = _run(L, variant, 32, q, A, Bv)
        assert int(got[0]) == 30439 and hist[k] == 1, (variant, hist)


def test_limits_rejected(L):
    import torch
    x = torch.zeros(256, dtype=torch.int64, device="cuda")
    h = torch.zeros(3, dtype=torch.int32, device="cuda")
    q29 = L.pm_ntt_primes(1024, 1, 29)[0]
    with pytest.raises(L.PMError):
        L.pm_reduce_apply(3, 32, x, x, x, h, q29)      # Alg. 3 needs len(q) <= 28 on 32-bit words
    with pytest.raises(L.PMError):
        L.pm_reduce_apply(4, 32, x, x, x, h, (1 << 31) + 11)
