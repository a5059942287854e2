"""Squint at insertion and the GPU FIFO replay of squinted transitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Alg. 1 downsamples every observation as it is observed and stores the
downsampled observation and next observation, with proprio, action and reward,
in the replay buffer; Sec. V (Replay Buffer Size) holds that buffer on the GPU
as a simple FIFO, which the small 16 x 16 frames make affordable.

Readings (the paper fixes neither the stored type nor the ring mechanics):
  * a stored frame is the k x k block mean of the raw uint8 frame rounded to the
    nearest integer, ties to even, kept as uint8 in HWC order at the squinted
    size (H/k, W/k, C).  The networks then see q / 255 - 0.5, which is the
    squint of that stored frame with k = 1.
  * FIFO: the i-th of n transitions inserted while the write position is p
    lands in row (p + i) mod capacity; afterwards p <- (p + n) mod capacity and
    size <- min(size + n, capacity).  One insertion holds at most `capacity`
    transitions.
Pinned by: exact rational means rounded by Python's round-half-even, constant
frames, the k = 1 identity, a deque model of the FIFO, and an update from a ring
of block-constant frames that must equal the update from the raw frames (tests).
"""
import numpy as np

from .squint import block_sums

FIELDS = ("obs", "next_obs", "proprio", "next_proprio", "action", "reward", "done")


def squint_u8(frames, k):
    """[n, H, W, C] uint8 -> [n, H/k, W/k, C] uint8 block means, nearest, ties to even."""
    s = block_sums(frames, k)                      # [n, C, h, w] exact int64
    kk = k * k
    q, r = np.divmod(s, kk)
    q = q + ((2 * r > kk) | ((2 * r == kk) & (q % 2 == 1)))
    return np.ascontiguousarray(q.transpose(0, 2, 3, 1)).astype(np.uint8)


class Ring:
    """Host model of the device ring: storage, write position and size."""

    def __init__(self, capacity, side, C, proprio, action):
        self.cap, self.pos, self.size = int(capacity), 0, 0
        self.obs = np.zeros((capacity, side, side, C), np.uint8)
        self.next_obs = np.zeros((capacity, side, side, C), np.uint8)
        self.proprio = np.zeros((capacity, proprio), np.float32)
        self.next_proprio = np.zeros((capacity, proprio), np.float32)
        self.action = np.zeros((capacity, action), np.float32)
        self.reward = np.zeros(capacity, np.float32)
        self.done = np.zeros(capacity, np.uint8)

    def insert(self, k, obs, next_obs, proprio, next_proprio, action, reward, done):
        n = len(obs)
        assert n <= self.cap
        rows = (self.pos + np.arange(n)) % self.cap
        self.obs[rows] = squint_u8(obs, k)
        self.next_obs[rows] = squint_u8(next_obs, k)
        self.proprio[rows] = proprio
        self.next_proprio[rows] = next_proprio
        self.action[rows] = action
        self.reward[rows] = reward
        self.done[rows] = done
        self.pos = (self.pos + n) % self.cap
        self.size = min(self.size + n, self.cap)

    def replay(self):
        """The replay dict the update reads: stored frames are squinted, so k = 1."""
        out = {f: getattr(self, f) for f in FIELDS}
        out["size"] = self.size
        out["k"] = 1
        return out
