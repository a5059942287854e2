"""Synthetic GPU environment stub for the environment-step loop of Alg. 1.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Alg. 1's outer loop observes, acts, steps the simulator and stores the
transition before the UTD updates.  The paper's simulator (ManiSkill3 with
batched rendering) is not available; this stub stands in for it with a
deterministic point-mass task and a cheap integer renderer, so the loop's data
path (act -> step -> insert -> updates) runs end to end on the device.

Definition (both sides implement it; frames are bit-exact, rewards FP32):
  state per env: proprio s[P] (FP32), goal g[2], step t, episode number, and the
  pixel positions of the last three frames (the frame stack)
  reset (episode ep): Philox4x32-10 words w of counters (env, 5, ep, q), q = 0..3,
    key = seed: s_j = 0.5 (2 u(w_j) - 1) for j < P (words in order), g_i = 1.5
    (2 u(w_{12+i}) - 1), u(w) = ((w >> 9) + 0.5) 2^-23; t = 0; stack = 3 copies
    of pix(s)
  step with action a[A]: s_j <- clamp(s_j + a_{j mod A} / 8, -2, 2);
    reward = -((s_0 - g_0)^2 + (s_1 - g_1)^2); t <- t + 1; done = (t == T);
    stack <- (pix(s), previous two); next frame rendered from the stack; when
    done, the env resets (episode + 1) and the observation for the next step is
    the reset frame, else it is the next frame
  pix(s) = clamp(floor(H/2 + (H/8) s_0), 0, H-1), same for s_1 with W
  render: slot k (0 = newest) fills channels 3k..3k+2; a pixel within radius
    H/8 of the slot's position (dx^2 + dy^2 <= (H/8)^2) takes (200, 120, 40),
    other pixels ((x xor y) * 5 + 11 c) mod 64
Pinned by: a brute-force per-pixel renderer, the clamp bounds, episode length
and reset determinism (tests).
"""
import numpy as np

from .philox import philox4x32_10

COLOR = (200, 120, 40)


def _u(w):
    return ((w >> 9).astype(np.float32) + np.float32(0.5)) * np.float32(2.0 ** -23)


def pix(v, side):
    q = np.floor(np.float32(side // 2) + np.float32(side // 8) * v.astype(np.float32))
    return np.clip(q, 0, side - 1).astype(np.int64)


def render(stack, H, W, C):
    """stack [n, 3, 2] (x, y) pixel positions -> frames [n, H, W, C] uint8."""
    n = stack.shape[0]
    y = np.arange(H)[:, None, None]
    x = np.arange(W)[None, :, None]
    c = np.arange(C)[None, None, :]
    bg = (((x ^ y) * 5 + 11 * c) % 64).astype(np.uint8)
    out = np.broadcast_to(bg, (n, H, W, C)).copy()
    R2 = (H // 8) ** 2
    for k in range(C // 3):
        dx = np.arange(W)[None, None, :] - stack[:, k, 0][:, None, None]
        dy = np.arange(H)[None, :, None] - stack[:, k, 1][:, None, None]
        inside = dx * dx + dy * dy <= R2
        for rgb in range(3):
            ch = out[:, :, :, 3 * k + rgb]
            ch[inside] = COLOR[rgb]
    return out


class Env:
    def __init__(self, n, H, W, C, P, A, T, seed):
        assert 2 <= P <= 12 and C in (3, 6, 9)
        self.n, self.H, self.W, self.C, self.P, self.A, self.T = n, H, W, C, P, A, T
        self.k0, self.k1 = np.uint32(seed & 0xFFFFFFFF), np.uint32(seed >> 32)
        self.s = np.zeros((n, P), np.float32)
        self.g = np.zeros((n, 2), np.float32)
        self.t = np.zeros(n, np.int64)
        self.ep = np.zeros(n, np.int64)
        self.stack = np.zeros((n, 3, 2), np.int64)
        for e in range(n):
            self._reset(e)
        self.obs = render(self.stack, H, W, C)

    def _reset(self, e):
        w = []
        for q in range(4):
            w += list(philox4x32_10(e, 5, self.ep[e], q, self.k0, self.k1))
        w = np.array(w, dtype=np.uint32)
        self.s[e] = np.float32(0.5) * (np.float32(2.0) * _u(w[:self.P]) - np.float32(1.0))
        self.g[e] = np.float32(1.5) * (np.float32(2.0) * _u(w[12:14]) - np.float32(1.0))
        self.t[e] = 0
        p = np.array([pix(self.s[e, 0:1], self.W)[0], pix(self.s[e, 1:2], self.H)[0]])
        self.stack[e] = p[None, :]

    def step(self, action):
        """Returns the transition (obs, proprio, reward, next_obs, next_proprio, done)
        and advances the observation (reset frames where episodes ended)."""
        a = np.asarray(action, np.float32)
        obs, prop = self.obs, self.s.copy()
        cols = np.arange(self.P) % self.A
        self.s = np.clip(self.s + a[:, cols] / np.float32(8.0), np.float32(-2.0), np.float32(2.0))
        d0 = self.s[:, 0].astype(np.float64) - self.g[:, 0]
        d1 = self.s[:, 1].astype(np.float64) - self.g[:, 1]
        reward = -(d0 * d0 + d1 * d1)
        self.t += 1
        done = (self.t == self.T).astype(np.uint8)
        newest = np.stack([pix(self.s[:, 0], self.W), pix(self.s[:, 1], self.H)], axis=1)
        self.stack = np.concatenate([newest[:, None, :], self.stack[:, :2]], axis=1)
        next_obs = render(self.stack, self.H, self.W, self.C)
        next_prop = self.s.copy()
        for e in np.nonzero(done)[0]:
            self.ep[e] += 1
            self._reset(e)
        self.obs = render(self.stack, self.H, self.W, self.C)
        return dict(obs=obs, proprio=prop, action=a, reward=reward, next_obs=next_obs, next_proprio=next_prop,
                    done=done)
