"""The float comparison of the parity tests: bit for bit, NaN payloads aside."""
import numpy as np

from gpu_common import same_floats


def test_same_floats_is_bitwise_but_ignores_nan_payloads():
    pos_nan = np.array([0x7FC00000], np.uint32).view(np.float32)
    neg_nan = np.array([0xFFC00000], np.uint32).view(np.float32)
    assert same_floats(np.r_[1.0, pos_nan], np.r_[1.0, neg_nan])
    assert not same_floats(np.float32([0.0]), np.float32([-0.0]))
    assert not same_floats(np.float32([1.0]), np.nextafter(np.float32([1.0]), np.float32(2)))
    assert not same_floats(np.r_[np.float32(1.0), pos_nan], np.float32([1.0, 1.0]))
    assert not same_floats(np.float32([1.0]), np.float32([1.0, 1.0]))
