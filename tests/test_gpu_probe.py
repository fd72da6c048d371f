"""The library's VALU issue-cost probe (a measurement aid for the ALU
rooflines): every op reports a positive cycle count per wave64 instruction
in a plausible range, and the C ABI rejects bad arguments."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_2011_04130_amd as q
    c = q.Context(0)
    yield c
    c.close()


def test_issue_rates(ctx):
    r = ctx.issue_rates(2.4)
    assert list(r) == ["v_add_u32", "v_sub_u32", "v_min_u32", "v_xor_b32", "v_mul_lo_u32",
                       "v_mul_hi_u32", "v_mad_u64_u32", "v_bitop3_b32"]
    for name, cyc in r.items():
        assert 0.5 < cyc < 64.0, (name, cyc)


def test_issue_rates_rejects_bad_arguments(ctx):
    lib = ctx._lib
    buf = (ctypes.c_double * 8)()
    einval = -1  # QRNG_EINVAL
    assert lib.qrng_profile_issue_rates(ctx._h, 0.0, buf, 8, None) == einval
    assert lib.qrng_profile_issue_rates(None, 2.4, buf, 8, None) == einval
    assert lib.qrng_profile_issue_op_name(8) is None
    assert lib.qrng_profile_issue_op_name(-1) is None
