"""Pins of the oracle's squint (area downsampling)."""
import numpy as np

from oracle import squint


def _brute(frames, k):
    n, H, W, C = frames.shape
    out = np.zeros((n, C, H // k, W // k), dtype=np.int64)
    for b in range(n):
        for c in range(C):
            for y in range(H // k):
                for x in range(W // k):
                    s = 0
                    for i in range(k):
                        for j in range(k):
                            s += int(frames[b, k * y + i, k * x + j, c])
                    out[b, c, y, x] = s
    return out


def test_block_sum_brute_force():
    rng = np.random.default_rng(0)
    for (H, k, C) in ((32, 2, 3), (64, 4, 9), (24, 3, 2)):
        f = rng.integers(0, 256, size=(2, H, H, C), dtype=np.uint8)
        np.testing.assert_array_equal(squint.block_sums(f, k), _brute(f, k))


def test_identity_and_constant():
    rng = np.random.default_rng(1)
    f = rng.integers(0, 256, size=(3, 16, 16, 9), dtype=np.uint8)
    np.testing.assert_array_equal(squint.block_sums(f, 1), f.transpose(0, 3, 1, 2))
    np.testing.assert_allclose(squint.squint(f, 1), f.transpose(0, 3, 1, 2) / 255.0 - 0.5, rtol=0, atol=0)
    const = np.full((1, 64, 64, 9), 200, dtype=np.uint8)
    assert np.all(squint.squint(const, 4) == 200 / 255.0 - 0.5)
    assert np.all(squint.squint(np.zeros((1, 32, 32, 3), np.uint8), 2) == -0.5)
    assert np.all(squint.squint(np.full((1, 32, 32, 3), 255, np.uint8), 2) == 0.5)


def test_fp32_rounding_is_ieee_per_element():
    rng = np.random.default_rng(2)
    f = rng.integers(0, 256, size=(2, 64, 64, 9), dtype=np.uint8)
    s = _brute(f, 4)
    x32 = squint.squint_f32(f, 4)
    assert x32.dtype == np.float32
    for v, got in zip(s.ravel()[:500], x32.ravel()[:500]):
        q = np.float32(np.float32(v) / np.float32(255 * 16))
        assert np.float32(q - np.float32(0.5)) == got
    # the FP32 value is within one FP32 rounding of the FP64 value
    np.testing.assert_allclose(x32, squint.squint(f, 4), rtol=0, atol=2 ** -24)
