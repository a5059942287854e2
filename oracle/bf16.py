"""bfloat16 operand emulation for the oracle's `bf16_operands` mode.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The mixed-precision form of the update (Sec. IV, PyTorch optimisations:
bfloat16 autocast of the update loop) multiplies bfloat16 operands and
accumulates in a wider type.  The oracle reproduces that by rounding each GEMM
or convolution operand to the nearest bfloat16 value (ties to even) and then
multiplying in FP64.  bfloat16 has FP32's exponent range and an 8-bit
significand (7 stored bits plus the implicit one).
Pinned by: exhaustive agreement with torch's float32->bfloat16 cast on values
that are exactly float32, and the tie-to-even special cases (tests).
"""
import numpy as np

_MIN_NORMAL = 2.0 ** -126
_SUB_QUANTUM = 2.0 ** -133


def round_bf16(x):
    """Round FP64 values to the nearest bfloat16 value, ties to even (as FP64)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m * 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.round(m * 256.0), e - 8)  # 8 significant bits, half-even
    small = np.abs(x) < _MIN_NORMAL
    if np.any(small):
        r = np.where(small, np.round(x / _SUB_QUANTUM) * _SUB_QUANTUM, r)
    return r


def maybe(x, on):
    """A parameter operand: rounded to bfloat16 in the bfloat16-operand mode."""
    return round_bf16(x) if on else x


# Sensitivity hook, off (None) in every ordinary run.  The tests' measurement of
# the oracle's own bfloat16-mode sensitivity sets it to a function that scales a
# computed operand by (1 + delta s) before it is rounded; parameter operands are
# never perturbed (both sides round the same FP32 parameter values).
_computed_perturbation = None


def set_computed_perturbation(fn):
    global _computed_perturbation
    _computed_perturbation = fn


def maybe_computed(x, on):
    """A computed operand (activation or upstream gradient): rounded to bfloat16
    in the bfloat16-operand mode."""
    if on and _computed_perturbation is not None:
        x = _computed_perturbation(np.asarray(x, dtype=np.float64))
    return round_bf16(x) if on else x
