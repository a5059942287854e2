"""Pins of the oracle's synthetic environment stub."""
import numpy as np

from oracle import env


def _brute_render(stack, H, W, C):
    out = np.zeros((len(stack), H, W, C), np.uint8)
    R2 = (H // 8) ** 2
    for n in range(len(stack)):
        for y in range(H):
            for x in range(W):
                for c in range(C):
                    k = c // 3
                    px, py = stack[n][k]
                    if (x - px) ** 2 + (y - py) ** 2 <= R2:
                        out[n, y, x, c] = env.COLOR[c % 3]
                    else:
                        out[n, y, x, c] = ((x ^ y) * 5 + 11 * c) % 64
    return out


def test_render_matches_per_pixel_loops():
    rng = np.random.default_rng(0)
    stack = rng.integers(0, 16, size=(3, 3, 2))
    stack[0, 1] = (0, 15)         # discs clipped by the border
    np.testing.assert_array_equal(env.render(stack, 16, 16, 6 + 3), _brute_render(stack, 16, 16, 9))


def test_dynamics_bounds_episodes_and_resets():
    n, T = 5, 7
    e = env.Env(n, 32, 32, 9, 12, 6, T, seed=11)
    twin = env.Env(n, 32, 32, 9, 12, 6, T, seed=11)
    assert np.all(np.abs(e.s) <= 0.5) and np.all(np.abs(e.g) <= 1.5)
    rng = np.random.default_rng(1)
    for step in range(3 * T):
        a = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
        s0 = e.s.copy()
        tr = e.step(a)
        twin.step(a)
        want = np.clip(s0 + a[:, np.arange(12) % 6] / 8, -2, 2)
        np.testing.assert_array_equal(tr["next_proprio"], want)
        np.testing.assert_array_equal(tr["proprio"], s0)
        assert np.all(tr["done"] == ((step + 1) % T == 0))
        assert np.all(tr["reward"] <= 0)
        # the newest stack slot marks the post-step position
        px = np.clip(np.floor(16 + 4 * want[:, 0]), 0, 31).astype(int)
        py = np.clip(np.floor(16 + 4 * want[:, 1]), 0, 31).astype(int)
        assert np.all(tr["next_obs"][np.arange(n), py, px, 0] == env.COLOR[0])
        if tr["done"][0]:
            assert np.all(e.t == 0) and np.all(np.abs(e.s) <= 0.5)
            assert not np.array_equal(e.s, want)
        np.testing.assert_array_equal(e.obs, twin.obs)     # deterministic given the seed
    big = env.Env(2, 32, 32, 3, 2, 2, 1000, seed=3)
    for _ in range(40):
        big.step(np.ones((2, 2), np.float32))
    assert np.all(big.s == 2.0)                            # the clamp holds
