"""Philox4x32-10 counter-based RNG and the draws the update makes from it.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Philox4x32-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter is mixed by ten
rounds of two 32x32->64 multiplies, with a 2x32-bit key advanced by the
Weyl constants between rounds.

Uses in the update (Alg. 1 draws each minibatch from the replay buffer; the
sampling law is unstated and read as uniform with replacement; Eq. (1) and
Eq. (3) need reparameterised actions drawn from the stochastic policy):
  replay index   idx[b] = mulhi32(w0, size), counter (u, 0, b, 0), key = seed
  Gaussian noise stream s in {1, 2}, element e: counter (u, s, e, 0);
                 Box-Muller on words w0, w1 with uniforms ((w >> 9) + 0.5) / 2^23
                 (23 random bits plus a half: exact in FP32, strictly inside (0, 1))
  act() sample   element e = row*A + d of a request: counter (e, 3, id_lo, id_hi),
                 so a row's noise depends only on (request id, row), not on batching
Pinned by: rocRAND's host-side Philox4x32-10 engine, a second scalar
implementation on Python ints, and a chi-square uniformity check (tests).
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 arrays; returns four uint32 arrays."""
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [v.astype(np.uint32) for v in c]


def philox4x32_10_scalar(ctr, key):
    """Second, independent implementation on Python ints (used to pin the first)."""
    x = list(ctr)
    k = list(key)
    for r in range(10):
        if r:
            k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
        a = M0 * x[0]
        b = M1 * x[2]
        x = [((b >> 32) ^ x[1] ^ k[0]) & MASK, b & MASK,
             ((a >> 32) ^ x[3] ^ k[1]) & MASK, a & MASK]
    return tuple(x)


def _key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK, seed >> 32


def sample_indices(seed, update, size, n):
    """Uniform replay indices with replacement in [0, size): mulhi32(w0, size)."""
    k0, k1 = _key(seed)
    b = np.arange(n, dtype=np.uint64)
    w = philox4x32_10(np.full(n, update), 0, b, 0, k0, k1)
    return ((w[0].astype(np.uint64) * np.uint64(size)) >> np.uint64(32)).astype(np.int64)


def _uniform23(w):
    """(w >> 9) + 0.5 scaled by 2^-23: strictly inside (0, 1), exact in FP32."""
    return ((w.astype(np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(w0, w1):
    u1 = _uniform23(w0)
    u2 = _uniform23(w1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def gaussian(seed, update, stream, n):
    """n standard normals of noise stream `stream` for update `update` (FP64)."""
    k0, k1 = _key(seed)
    e = np.arange(n, dtype=np.uint64)
    w = philox4x32_10(np.full(n, update), stream, e, 0, k0, k1)
    return box_muller(w[0], w[1])


def act_noise(seed, request_id, rows, action_dim):
    """Sampling noise of act(): row-major [rows, action_dim], keyed by request id."""
    k0, k1 = _key(seed)
    rid = int(request_id) & 0xFFFFFFFFFFFFFFFF
    e = np.arange(rows * action_dim, dtype=np.uint64)
    w = philox4x32_10(e, 3, rid & MASK, rid >> 32, k0, k1)
    return box_muller(w[0], w[1]).reshape(rows, action_dim)
