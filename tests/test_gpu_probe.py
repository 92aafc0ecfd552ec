"""The VALU issue-rate probe behind the roofline's peak: every instruction class
measured, rates and the loaded shader clock in a physically possible range."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_valu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2209_01290_amd import lib
    rates, mhz = lib.pm_probe_valu()
    assert set(rates) == {"v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_alignbit_b32", "v_add3_u32",
                          "v_sub_co_u32", "v_lshl_add_u64", "v_add_u32", "v_xor_b32", "v_mov_b32"}
    assert 500.0 < mhz < 3500.0, mhz
    for name, r in rates.items():
        assert 1e12 < r < 2e14, (name, r)
