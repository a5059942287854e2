"""Shared helpers of the GPU parity tests (inputs come from the synthetic
generators; expected values only from oracle/)."""
import json
import os

import numpy as np
import torch

from oracle import layout as olayout
from paper_2602_21203_amd import configs, synthetic

LOSS_RTOL, LOSS_ATOL = 1e-4, 1e-6      # losses: |d| <= 1e-4 |ref| + 1e-6
GRAD_RTOL = 1e-3                       # gradients: ||d||_2 <= 1e-3 ||ref||_2 per tensor
ACT_RTOL = 1e-3                        # act(): ||d||_2 <= 1e-3 ||ref||_2 over the action array

# BF16 against the oracle's bfloat16-operand mode.  Both sides round the same
# operands, but the value being rounded is FP32 on the GPU and FP64 in the
# oracle, so a few rounding decisions differ and later decisions of those rows
# follow.  How far each result moves through such flips is measured on the
# oracle alone (tests/sensitivity.py, stored in golden/bf16_sensitivity.json by
# golden/make_bf16_sensitivity.py): every computed operand that FP32 cannot hold
# exactly is moved by delta = 2^-22 times the rms of its row (random sign), the
# size of the FP32 path's own deviation from FP64, before it is rounded; the
# mean change over 8 draws is the sensitivity.  Each BF16 tolerance is
# max(stated bar, SENS_FACTOR x that sensitivity), per gradient tensor and per
# statistic.
SENS_FACTOR = 2.0
_SENS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bf16_sensitivity.json")
with open(_SENS_PATH) as _f:
    SENS = json.load(_f)


def bf16_grad_tol(case, tensor):
    return max(GRAD_RTOL, SENS_FACTOR * SENS["cases"][case]["grad"][tensor])


def bf16_stat_tol(case, stat):
    return max(LOSS_RTOL, SENS_FACTOR * SENS["cases"][case]["stat"][stat])


def bf16_enc_op_tol(case, what):
    """Encoder op parity (features or a gradient tensor) in the bfloat16 mode."""
    return max(GRAD_RTOL, SENS_FACTOR * SENS["enc_ops"][case][what])


def bf16_act_tol(kind):
    return max(ACT_RTOL, SENS_FACTOR * SENS["act"][kind])


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


def assert_loss(got, ref, what="", scale=None, rtol=LOSS_RTOL):
    """|got - ref| <= rtol * scale + 1e-6, scale = |ref| unless the statistic is a
    mean of signed terms, whose magnitude (the oracle's stat_scale) sets the scale."""
    s = abs(ref) if scale is None else max(abs(ref), scale)
    assert abs(got - ref) <= rtol * s + LOSS_ATOL, f"{what}: got {got!r} ref {ref!r} scale {s!r}"


def stat_rtol(prec, name, case=None):
    """Tolerance of an update statistic against the oracle in the same precision mode."""
    return LOSS_RTOL if prec == 0 else bf16_stat_tol(case, name)


def assert_grads_per_tensor(got_flat, ref_flat, name, base, lo, hi, rtol=GRAD_RTOL, case=None, dims=None):
    """Per-tensor relative-norm check of flat gradient slices [lo, hi) (offsets
    absolute).  With `case` (BF16), each tensor's tolerance comes from the
    measured sensitivity of that case; otherwise it is `rtol`.  Returns the worst
    (error, tolerance, tensor) by error / tolerance."""
    tab = olayout.offsets(dims if dims is not None else odims(name))[0]
    bad = []
    worst = (0.0, rtol, "")
    for n, (o, s) in tab.items():
        if o < lo or o >= hi:
            continue
        k = int(np.prod(s))
        g = got_flat[o - base:o - base + k]
        r = ref_flat[o - lo:o - lo + k]
        e = rel_norm(g, r)
        tol = bf16_grad_tol(case, n) if case is not None else rtol
        if e / tol > worst[0] / worst[1]:
            worst = (e, tol, n)
        if e > tol:
            bad.append((n, e, tol))
    assert not bad, f"gradient tensors over tolerance (tensor, error, tolerance): {bad}"
    return worst
