"""How the matrix instructions accumulate (GPU): the property the parity tolerances model.

The oracle's error model (conet64._conv_acc, used only for tolerances) says: the FP8
instructions (16x16x128 and 32x32x64 e4m3) keep a product whole if it is at least 2^-B of the
largest product of its group of 8 consecutive K values (B = conet64.FP8_MFMA_GROUP_BITS) and
drop a smaller one, while products in other groups, and BF16 products, are kept to FP32
resolution. Checked here through conet_mfma_dot on one instruction with crafted operands: a
product of 256 at k = 0 and seven equal small products in the same or in the next group.
"""
import numpy as np
import pytest

from oracle import conet64 as o

pytestmark = pytest.mark.gpu

B = o.FP8_MFMA_GROUP_BITS


def _e4m3_pow2(e: int) -> int:
    """e4m3fn code of 2^e (normal for e >= -6, subnormal down to 2^-9)."""
    return (e + 7) << 3 if e >= -6 else 1 << (e + 9)


def _fp8_sum(shape, ratio_exp, first):
    from paper_2510_12739_amd import mfma_dot
    K = 128 if shape == 16 else 64
    a = np.zeros(K, np.uint8)
    b = np.zeros(K, np.uint8)
    a[0], b[0] = _e4m3_pow2(8), _e4m3_pow2(0)            # 256
    e = 8 - ratio_exp                                     # small product 2^e = 256 * 2^-ratio_exp
    ea = max(e, -9)
    a[first:first + 7], b[first:first + 7] = _e4m3_pow2(ea), _e4m3_pow2(e - ea)
    return mfma_dot("fp8", shape, a, b), 2.0 ** e


@pytest.mark.parametrize("shape", [16, 32])
def test_fp8_group_truncation(shape):
    kept, s = _fp8_sum(shape, B, 1)                       # same group: 2^-B of the largest is kept
    assert kept == np.float32(256.0 + 7 * s)
    dropped, s = _fp8_sum(shape, B + 1, 1)                # same group: 2^-(B+1) is dropped
    assert dropped == np.float32(256.0)
    other, s = _fp8_sum(shape, B + 1, 8)                  # next group: kept
    assert other == np.float32(256.0 + 7 * s)


@pytest.mark.parametrize("shape", [16, 32])
def test_bf16_products_keep_fp32_resolution(shape):
    from paper_2510_12739_amd import mfma_dot
    K = 32 if shape == 16 else 16
    for ratio_exp in (16, 20, 23):
        a = np.zeros(K, np.float32)
        b = np.zeros(K, np.float32)
        a[0], b[0] = 256.0, 1.0
        a[1:8], b[1:8] = 1.0, 2.0 ** (8 - ratio_exp)
        got = mfma_dot("bf16", shape, a, b)
        assert got == np.float32(256.0 + 7 * 2.0 ** (8 - ratio_exp)), (shape, ratio_exp, got)
