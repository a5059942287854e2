"""Shared helpers of the GPU parity tests (inputs come from the synthetic
generators; expected values only from oracle/)."""
import numpy as np
import torch

from oracle import layout as olayout
from paper_2602_21203_amd import configs, synthetic

LOSS_RTOL, LOSS_ATOL = 1e-4, 1e-6      # losses: |d| <= 1e-4 |ref| + 1e-6
GRAD_RTOL = 1e-3                       # gradients: ||d||_2 <= 1e-3 ||ref||_2 per tensor
# bfloat16 operands against the oracle's bfloat16-operand mode: both sides round
# the same operands, but the value being rounded is FP32 on the GPU and FP64 in
# the oracle, so a few rounding decisions differ, and a row whose input differs
# by one bfloat16 unit has its later decisions decorrelated.  Tensors at the end
# of the longest chain (the encoder, after the critic backward) therefore carry
# up to about one bfloat16 unit roundoff of relative difference.
GRAD_RTOL_BF16 = 2.0 ** -8


def cfg(name):
    return configs.CONFIGS[name]


def odims(name):
    return olayout.dims(**cfg(name))


def table(name):
    return [(n, o, s) for n, (o, s) in olayout.offsets(odims(name))[0].items()]


def params(name, seed=1):
    return synthetic.init_params(table(name), seed=seed)


def np_replay(rep):
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in rep.items()}
    return out


def rel_norm(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30))


def assert_loss(got, ref, what="", scale=None):
    """|got - ref| <= 1e-4 * scale + 1e-6, scale = |ref| unless the statistic is a
    mean of signed terms, whose magnitude (the oracle's stat_scale) sets the scale."""
    s = abs(ref) if scale is None else max(abs(ref), scale)
    assert abs(got - ref) <= LOSS_RTOL * s + LOSS_ATOL, f"{what}: got {got!r} ref {ref!r} scale {s!r}"


def assert_grads_per_tensor(got_flat, ref_flat, name, base, lo, hi, rtol=GRAD_RTOL):
    """Per-tensor relative-norm check of flat gradient slices [lo, hi) (offsets absolute)."""
    tab = olayout.offsets(odims(name))[0]
    bad = []
    worst = 0.0
    for n, (o, s) in tab.items():
        if o < lo or o >= hi:
            continue
        k = int(np.prod(s))
        g = got_flat[o - base:o - base + k]
        r = ref_flat[o - lo:o - lo + k]
        e = rel_norm(g, r)
        worst = max(worst, e)
        if e > rtol:
            bad.append((n, e))
    assert not bad, f"gradient tensors over tolerance {rtol}: {bad}"
    return worst
