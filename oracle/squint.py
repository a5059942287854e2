"""Resolution squinting: area downsampling of uint8 camera frames.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. IV (Resolution Squinting) renders at a high resolution and area
downsamples to 16x16; Alg. 1 applies the downsampling to every observation
before it reaches the networks.  Area downsampling by an integer factor k is
the mean over each disjoint k x k block.  Frames are HWC uint8 (channel
c = 3*s + rgb for stack slot s); the output is CHW, scaled to [-0.5, 0.5]:
    S[c, y, x] = sum_{i, j < k} frame[k*y + i, k*x + j, c]   (exact integer)
    x = S / (255 k^2) - 0.5
Pinned by: a brute-force nested-loop block sum, k = 1 identity and constant
frames (tests).
"""
import numpy as np


def block_sums(frames, k):
    """Exact integer k x k block sums: [n, H, W, C] uint8 -> [n, C, H/k, W/k] int64."""
    f = np.asarray(frames)
    n, H, W, C = f.shape
    assert H % k == 0 and W % k == 0
    s = f.astype(np.int64).reshape(n, H // k, k, W // k, k, C).sum(axis=(2, 4))
    return np.ascontiguousarray(s.transpose(0, 3, 1, 2))


def squint(frames, k):
    """FP64 scaled block means in [-0.5, 0.5]."""
    return block_sums(frames, k) / (255.0 * k * k) - 0.5


def squint_f32(frames, k):
    """The same value evaluated in IEEE FP32: fl(fl(S / (255 k^2)) - 0.5)."""
    s = block_sums(frames, k).astype(np.float32)
    return s / np.float32(255 * k * k) - np.float32(0.5)
