"""Pins of the oracle's squint at insertion and FIFO replay ring."""
from collections import deque
from fractions import Fraction

import numpy as np

from oracle import ring, sac
from tests import helpers as H


def _brute_u8(frames, k):
    n, Hh, W, C = frames.shape
    out = np.zeros((n, Hh // k, W // k, C), np.uint8)
    for b in range(n):
        for y in range(Hh // k):
            for x in range(W // k):
                for c in range(C):
                    s = sum(int(frames[b, k * y + i, k * x + j, c]) for i in range(k) for j in range(k))
                    out[b, y, x, c] = round(Fraction(s, k * k))   # nearest, ties to even
    return out


def test_squint_u8_brute_force_and_ties():
    rng = np.random.default_rng(3)
    for (Hh, k, C) in ((8, 2, 3), (16, 4, 2), (12, 3, 1)):
        f = rng.integers(0, 256, size=(2, Hh, Hh, C), dtype=np.uint8)
        np.testing.assert_array_equal(ring.squint_u8(f, k), _brute_u8(f, k))
        # small values make exact halves common
        f = rng.integers(0, 3, size=(2, Hh, Hh, C), dtype=np.uint8)
        np.testing.assert_array_equal(ring.squint_u8(f, k), _brute_u8(f, k))
    # hand-made ties with k = 2: means 0.5 -> 0, 1.5 -> 2, 2.5 -> 2, 254.5 -> 254
    blocks = [(0, 1, 0, 1), (1, 2, 1, 2), (2, 3, 2, 3), (254, 255, 254, 255), (3, 3, 3, 4)]
    f = np.zeros((1, 2, 2 * len(blocks), 1), np.uint8)
    for i, (a, b, c, d) in enumerate(blocks):
        f[0, 0, 2 * i], f[0, 0, 2 * i + 1], f[0, 1, 2 * i], f[0, 1, 2 * i + 1] = a, b, c, d
    assert list(ring.squint_u8(f, 2)[0, 0, :, 0]) == [0, 2, 2, 254, 3]


def test_squint_u8_identity_and_constant():
    rng = np.random.default_rng(4)
    f = rng.integers(0, 256, size=(3, 16, 16, 9), dtype=np.uint8)
    np.testing.assert_array_equal(ring.squint_u8(f, 1), f)
    for v in (0, 17, 255):
        out = ring.squint_u8(np.full((1, 64, 64, 9), v, np.uint8), 4)
        assert out.shape == (1, 16, 16, 9) and np.all(out == v)


def _batch(rng, n, Hh, C, P, A, start):
    return dict(obs=rng.integers(0, 256, size=(n, Hh, Hh, C), dtype=np.uint8),
                next_obs=rng.integers(0, 256, size=(n, Hh, Hh, C), dtype=np.uint8),
                proprio=np.arange(start, start + n, dtype=np.float32)[:, None] * np.ones((1, P), np.float32),
                next_proprio=rng.standard_normal((n, P)).astype(np.float32),
                action=rng.uniform(-1, 1, (n, A)).astype(np.float32),
                reward=rng.uniform(0, 1, n).astype(np.float32),
                done=(rng.uniform(0, 1, n) < 0.3).astype(np.uint8))


def test_fifo_matches_deque_model():
    rng = np.random.default_rng(5)
    cap, k, Hh, C, P, A = 7, 2, 8, 3, 2, 3
    r = ring.Ring(cap, Hh // k, C, P, A)
    model = deque(maxlen=cap)
    total = 0
    for n in (3, 5, 0, 7, 1, 6, 2):
        b = _batch(rng, n, Hh, C, P, A, total)
        r.insert(k, **b)
        for i in range(n):
            model.append(dict(obs=ring.squint_u8(b["obs"][i:i + 1], k)[0],
                              next_obs=ring.squint_u8(b["next_obs"][i:i + 1], k)[0],
                              **{f: b[f][i] for f in ("proprio", "next_proprio", "action", "reward", "done")}))
        total += n
        assert r.size == len(model) == min(total, cap)
        assert r.pos == total % cap
        for j, t in enumerate(model):        # oldest first
            row = (r.pos - r.size + j) % cap
            for f in ring.FIELDS:
                np.testing.assert_array_equal(getattr(r, f)[row], t[f])


def test_update_from_block_constant_ring_equals_raw_update():
    """Frames whose k x k blocks are constant squint exactly, so an update that
    samples the ring (k = 1 on stored frames) must equal the update on the raw
    frames at the same rows."""
    name, B, cap = "tiny", 8, 64
    d = H.odims(name)
    cfg = H.cfg(name)
    k, C, side = d.k, cfg["C"], cfg["H"] // d.k
    rng = np.random.default_rng(6)

    def blocky(n):
        q = rng.integers(0, 256, size=(n, side, side, C), dtype=np.uint8)
        return np.repeat(np.repeat(q, k, axis=1), k, axis=2)

    raw = _batch(rng, cap, cfg["H"], C, cfg["proprio"], cfg["action"], 0)
    raw["obs"], raw["next_obs"] = blocky(cap), blocky(cap)
    raw["done"] = (rng.uniform(0, 1, cap) < 0.1).astype(np.uint8)
    r = ring.Ring(cap, side, C, cfg["proprio"], cfg["action"])
    r.insert(k, **raw)
    rep_raw = dict(raw, size=cap)
    hp = sac.hparams(d)
    p0 = H.params(name).astype(np.float64)
    st_a, st_b = sac.new_state(d, p0), sac.new_state(d, p0)
    out_a = sac.sac_update(st_a, rep_raw, d, hp, B)
    out_b = sac.sac_update(st_b, r.replay(), d, hp, B)
    np.testing.assert_array_equal(out_a["stats"], out_b["stats"])
    np.testing.assert_array_equal(st_a.params, st_b.params)
    # and a ring of general frames differs from the raw update only through rounding
    raw2 = dict(raw, obs=rng.integers(0, 256, size=raw["obs"].shape, dtype=np.uint8))
    r2 = ring.Ring(cap, side, C, cfg["proprio"], cfg["action"])
    r2.insert(k, **raw2)
    out_c = sac.sac_update(sac.new_state(d, p0), r2.replay(), d, hp, B)
    out_d = sac.sac_update(sac.new_state(d, p0), dict(raw2, size=cap), d, hp, B)
    assert np.all(np.isfinite(out_c["stats"]))
    assert not np.array_equal(out_c["stats"], out_d["stats"])
