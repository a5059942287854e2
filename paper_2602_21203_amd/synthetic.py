"""Seeded synthetic inputs: replay contents, initial parameters, noise-free data.

This module holds no arithmetic of the method.  It only draws the inputs that
both the GPU library and the CPU checker consume, so that the two sides see
identical data.  The simulator's wrist-camera renders are replaced by frames
with spatial structure plus noise at the paper's squint geometry.

Frame recipe: for every frame and channel, the sum of 8 Gaussian blobs
A * exp(-((x - cx)^2 + (y - cy)^2) / (2 s^2)) with A ~ U[0, 128),
cx, cy ~ U[0, W), s ~ U[W/16, W/4], plus U[0, 32) noise, clamped to [0, 255]
and floored to uint8; stored HWC.  Stacked frames have independent blobs.
Other fields: proprio and next proprio ~ N(0, 1), action ~ U[-1, 1],
reward ~ U[0, 1], done ~ Bernoulli(0.01) (uint8).
Parameters: W and b ~ U(+-1/sqrt(fan_in)), LayerNorm gain 1 and bias 0,
log alpha = log_alpha0; all values are exactly representable in FP32.
"""
import numpy as np
import torch

N_BLOBS = 8


def _frames_chunk(n, H, W, C, gen, device):
    f32 = dict(dtype=torch.float32, device=device)
    amp = torch.rand(n, C, N_BLOBS, generator=gen, **f32) * 128.0
    cx = torch.rand(n, C, N_BLOBS, generator=gen, **f32) * W
    cy = torch.rand(n, C, N_BLOBS, generator=gen, **f32) * H
    s = W / 16.0 + torch.rand(n, C, N_BLOBS, generator=gen, **f32) * (W / 4.0 - W / 16.0)
    xs = torch.arange(W, **f32)
    ys = torch.arange(H, **f32)
    gx = torch.exp(-((xs.view(1, 1, 1, W) - cx[..., None]) ** 2) / (2.0 * s[..., None] ** 2))
    gy = torch.exp(-((ys.view(1, 1, 1, H) - cy[..., None]) ** 2) / (2.0 * s[..., None] ** 2))
    gy = (gy * amp[..., None]).reshape(n * C, N_BLOBS, H).transpose(1, 2).contiguous()
    gx = gx.reshape(n * C, N_BLOBS, W).contiguous()
    img = torch.bmm(gy, gx).reshape(n, C, H, W)
    img = img + torch.rand(n, C, H, W, generator=gen, **f32) * 32.0
    img = torch.floor(img.clamp(0.0, 255.0)).to(torch.uint8)
    return img.permute(0, 2, 3, 1).contiguous()


def frames(n, H, W, C, seed=0, device="cpu", chunk=2048):
    """[n, H, W, C] uint8 synthetic frames."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((n, H, W, C), dtype=torch.uint8, device=device)
    for i in range(0, n, chunk):
        j = min(n, i + chunk)
        out[i:j] = _frames_chunk(j - i, H, W, C, gen, device)
    return out


def replay(capacity, H, W, C, proprio, action, seed=0, device="cpu", done_rate=0.01):
    """Full synthetic replay as a dict of torch tensors (size == capacity)."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) + 1)
    f32 = dict(dtype=torch.float32, device=device)
    rep = dict(
        obs=frames(capacity, H, W, C, seed=seed * 2 + 100, device=device),
        next_obs=frames(capacity, H, W, C, seed=seed * 2 + 101, device=device),
        proprio=torch.randn(capacity, proprio, generator=gen, **f32),
        next_proprio=torch.randn(capacity, proprio, generator=gen, **f32),
        action=torch.rand(capacity, action, generator=gen, **f32) * 2.0 - 1.0,
        reward=torch.rand(capacity, generator=gen, **f32),
        done=(torch.rand(capacity, generator=gen, **f32) < done_rate).to(torch.uint8),
    )
    rep["size"] = capacity
    return rep


def init_params(table, seed=1, log_alpha0=0.0):
    """Flat FP32 parameter vector from a layout table [(name, offset, shape), ...]."""
    table = list(table)
    shapes = {name: shape for name, _, shape in table}
    total = max(o + int(np.prod(s)) for _, o, s in table)
    rng = np.random.default_rng(seed)
    p = np.zeros(total, dtype=np.float32)
    for name, o, shape in table:
        n = int(np.prod(shape))
        if name.endswith(".ln.g"):
            p[o:o + n] = 1.0
        elif name.endswith(".ln.b"):
            p[o:o + n] = 0.0
        elif name == "log_alpha":
            p[o] = log_alpha0
        else:
            wshape = shapes[name[:-1] + "W"]
            bound = 1.0 / float(np.prod(wshape[1:])) ** 0.5
            p[o:o + n] = rng.uniform(-bound, bound, n).astype(np.float32)
    return p
