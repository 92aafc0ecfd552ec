"""The seeded input generator: published SplitMix64 test vector, range,
determinism and independence of streams."""
import numpy as np

from paper_2209_01290_amd import synth


def test_splitmix64_reference_vector():
    # SplitMix64 seeded with 0: the first output is 0xE220A8397B1DCDAF,
    # the second 0x6E789E6AA1B965F4 (state advances by the golden gamma).
    assert synth._mix_int(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert synth._mix_int(2 * 0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    w = synth.words(0, 2)     # counter mode over key 0 is the plain sequence
    assert [int(x) for x in w] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]


def test_range_and_determinism():
    for q in [2, 97, 12289, 2**60 - 2**14 + 1, 2**62 - 57]:
        k = synth.key(synth.SEED_BASE, 1, 2, 3, 0)
        v = synth.uniform_mod(k, 5000, q)
        assert v.dtype == np.uint64 and int(v.max()) < q
        assert np.array_equal(v, synth.uniform_mod(k, 5000, q))
    k0 = synth.key(synth.SEED_BASE, 0, 0, 0, 0)
    k1 = synth.key(synth.SEED_BASE, 0, 0, 0, 1)
    assert k0 != k1
    q = 2**60 - 2**14 + 1
    a, b = synth.uniform_mod(k0, 4096, q), synth.uniform_mod(k1, 4096, q)
    assert not np.array_equal(a, b)
    # roughly uniform: mean near q/2
    assert abs(float(a.astype(np.float64).mean()) / q - 0.5) < 0.03


def test_operands_shape():
    a, b = synth.operands(5, [97, 193], polys=3, N=16)
    assert a.shape == (2, 3, 16) and b.shape == (2, 3, 16)
    assert int(a[0].max()) < 97 and int(b[1].max()) < 193
