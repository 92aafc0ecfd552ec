"""Bit-exact parity of the interleaved (coefficient-major) batch layout with
the CPU oracle, through the C ABI: the batch of a limb is stored as an N x P
matrix, coefficient j of polynomial p at [j * P + p]. Operands are drawn in
the [limb][poly][N] layout by the shared seeded generator, transposed for the
device, and the device result is transposed back and compared word for word
with the oracle (tolerance zero)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import first_mismatch, operands, oracle_ntt_fwd, oracle_ntt_inv, oracle_polymul, oracle_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    lib.load()
    return lib


def _sync():
    import torch
    torch.cuda.synchronize()


def _eq(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, "%s: %s" % (what, msg)


def to_il(x):
    """[limb][poly][N] -> [limb][N][poly] (contiguous)."""
    return np.ascontiguousarray(np.transpose(x, (0, 2, 1)))


def from_il(x, shape):
    """device result [limb][N][poly] -> [limb][poly][N]."""
    Lb, P, N = shape
    return np.ascontiguousarray(np.transpose(x.reshape(Lb, N, P), (0, 2, 1)))


def _ws(L, N, limbs, polys):
    import torch
    n = L.pm_polymul_il_workspace_bytes(N, limbs, polys)
    return torch.empty(n // 8, dtype=torch.int64, device="cuda") if n else None


def _setup(L, log2n, limbs, polys, request, bits=60):
    N = 1 << log2n
    qs = L.pm_ntt_primes(N, limbs, bits)
    fw_o, iv_o = oracle_tables(qs, N)
    prm = L.Params(N, limbs, primes=qs)
    a, b = operands(N, qs, polys, request=request)
    return N, qs, fw_o, iv_o, prm, a, b


# polys: one (the layouts coincide), a ragged wave, several ragged workgroups
POLYS = [1, 3, 69, 300]


@pytest.mark.parametrize("polys", POLYS)
@pytest.mark.parametrize("log2n", list(range(1, 18)))
def test_ntt_il(L, log2n, polys):
    if log2n >= 15 and polys > 69:
        polys = 20                       # keep the oracle run short at large N
    limbs = 2
    N, qs, fw_o, iv_o, prm, a, _ = _setup(L, log2n, limbs, polys, 1100 + log2n)
    x = L.to_device(to_il(a))
    L.pm_ntt_fwd_il(x, N, limbs, polys, qs, prm.psi_br)
    _sync()
    _eq(from_il(L.to_host(x), a.shape), oracle_ntt_fwd(a, qs, fw_o), "ntt_fwd_il N=%d P=%d" % (N, polys))
    L.pm_ntt_inv_il(x, N, limbs, polys, qs, prm.psi_inv_br)
    _sync()
    _eq(from_il(L.to_host(x), a.shape), a, "roundtrip il N=%d P=%d" % (N, polys))
    y = L.to_device(to_il(a))
    L.pm_ntt_inv_il(y, N, limbs, polys, qs, prm.psi_inv_br)
    _sync()
    _eq(from_il(L.to_host(y), a.shape), oracle_ntt_inv(a, qs, iv_o), "ntt_inv_il N=%d P=%d" % (N, polys))


@pytest.mark.parametrize("polys", POLYS)
@pytest.mark.parametrize("log2n", list(range(1, 18)))
def test_polymul_il(L, log2n, polys):
    import torch
    if log2n >= 15 and polys > 69:
        polys = 20
    limbs = 2
    N, qs, fw_o, iv_o, prm, a, b = _setup(L, log2n, limbs, polys, 1200 + log2n)
    da, db = L.to_device(to_il(a)), L.to_device(to_il(b))
    dc = torch.empty_like(da)
    L.pm_polymul_il(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    _sync()
    got = from_il(L.to_host(dc), a.shape)
    _eq(got, oracle_polymul(a, b, qs, N, fw_o, iv_o), "polymul_il N=%d P=%d" % (N, polys))
    if N <= 256:
        o = oracle.default()
        assert np.array_equal(got[1, polys - 1], o.polymul_schoolbook(a[1, polys - 1], b[1, polys - 1], qs[1]))


@pytest.mark.parametrize("log2n", [6, 12, 16])
@pytest.mark.parametrize("alias", ["c=a", "c=b", "a=b", "a=b=c"])
def test_aliasing_il(L, log2n, alias):
    limbs, polys = 2, 5
    N, qs, fw_o, iv_o, prm, a, b = _setup(L, log2n, limbs, polys, 1300 + log2n)
    if alias.startswith("a=b"):
        b = a
    da, db = L.to_device(to_il(a)), L.to_device(to_il(b))
    if alias == "c=a":
        dc = da
    elif alias == "c=b":
        dc = db
    elif alias == "a=b":
        db = da
        dc = L.to_device(np.zeros_like(to_il(a)))
    else:
        db = dc = da
    L.pm_polymul_il(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    _sync()
    _eq(from_il(L.to_host(dc), a.shape), oracle_polymul(a, b, qs, N, fw_o, iv_o), "il %s N=%d" % (alias, N))


def test_il_matches_standard_layout_kind_any(L):
    """Moduli outside [2^33, 2^61) (the run-time-window instantiation), 70 limbs
    (two chunks): the interleaved product equals the standard-layout product."""
    import torch
    N, polys = 1 << 12, 4
    qs = (L.pm_ntt_primes(N, 35, 62) + L.pm_ntt_primes(N, 35, 31))
    limbs = len(qs)
    prm = L.Params(N, limbs, primes=qs)
    a, b = operands(N, qs, polys, request=1400)
    da, db = L.to_device(a), L.to_device(b)
    dc = torch.empty_like(da)
    ws = torch.empty(max(L.pm_polymul_workspace_bytes(N, limbs, polys) // 8, 1), dtype=torch.int64, device="cuda")
    L.pm_polymul(da, db, dc, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, ws)
    ia, ib = L.to_device(to_il(a)), L.to_device(to_il(b))
    ic = torch.empty_like(ia)
    L.pm_polymul_il(ia, ib, ic, N, limbs, polys, qs, prm.psi_br, prm.psi_inv_br, _ws(L, N, limbs, polys))
    _sync()
    std = L.to_host(dc).reshape(a.shape)
    _eq(from_il(L.to_host(ic), a.shape), std, "il vs standard, 70 mixed limbs")
    fw_o, iv_o = oracle_tables(qs[:1] + qs[-1:], N)
    sub = [0, limbs - 1]
    _eq(std[sub], oracle_polymul(a[sub], b[sub], [qs[0], qs[-1]], N, fw_o, iv_o), "standard vs oracle")
