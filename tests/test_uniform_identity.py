"""The identity behind the GPU's uniforms (CPU, exhaustive).

The device forms u = (2 (x >> 9) + 1) 2^-24 without an integer-to-float
conversion: the 23 bits x >> 9 become the mantissa of a float in [1, 2)
(bit pattern 0x3F800000 | (x >> 9)), and one FP32 subtraction of the float
1 - 2^-24 leaves u.  That subtraction is exact because u is representable, so
the device's uniforms equal the oracle's definition bit for bit.  This test
checks the identity for all 2^23 mantissas in IEEE single precision.
"""
import numpy as np


def test_mantissa_uniform_identity_is_exact():
    m = np.arange(1 << 23, dtype=np.uint32)
    one_minus = np.float32(1.0 - 2.0 ** -24)
    assert one_minus.view(np.uint32) == 0x3F7FFFFF
    u = (np.uint32(0x3F800000) | m).view(np.float32) - one_minus
    assert u.dtype == np.float32
    exact = (2.0 * m.astype(np.float64) + 1.0) * 2.0 ** -24
    assert np.array_equal(u.astype(np.float64), exact)
    assert u.min() > 0.0 and u.max() < 1.0
