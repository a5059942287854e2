"""The oracle's own bfloat16-mode sensitivity (tests/sensitivity.py), from which
the BF16 tolerances of the GPU parity tests are derived: the stored table
(golden/bf16_sensitivity.json) is reproduced by the oracle at full size (16x16
at B = 512 and B = 2048, 32x32 at B = 128), covers every BF16 parity case, and
the measurement's hook leaves every ordinary oracle run untouched."""
import json
import os

import numpy as np
import pytest

from oracle import bf16 as obf16
from tests import helpers as H
from tests import sensitivity

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bf16_sensitivity.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_table_covers_every_case_and_tensor():
    g = _golden()
    assert g["delta"] == sensitivity.DELTA and g["n_perturb"] == sensitivity.N_PERTURB
    assert set(g["cases"]) == set(sensitivity.CASES)
    from oracle import layout as olayout
    for name, case in sensitivity.CASES.items():
        _, d = sensitivity.case_dims(case)
        assert set(g["cases"][name]["grad"]) == set(olayout.offsets(d)[0]), name
        assert set(g["cases"][name]["stat"]) == set(sensitivity.STAT_NAMES), name
    assert set(g["act"]) >= {"mean", "sample"}
    assert set(g["enc_ops"]) == set(sensitivity.ENC_OP_CASES)


def test_hook_is_inert_when_off():
    x = np.random.default_rng(0).normal(size=1000)
    assert obf16._computed_perturbation is None
    np.testing.assert_array_equal(obf16.maybe_computed(x, True), obf16.round_bf16(x))
    np.testing.assert_array_equal(obf16.maybe_computed(x, False), x)


def test_tolerance_rule():
    g = _golden()
    c = g["cases"]["full_b512"]
    for n, s in c["grad"].items():
        assert H.bf16_grad_tol("full_b512", n) == max(H.GRAD_RTOL, H.SENS_FACTOR * s)
    assert H.bf16_stat_tol("full_b512", "critic_loss") == max(H.LOSS_RTOL, H.SENS_FACTOR * c["stat"]["critic_loss"])


@pytest.mark.parametrize("name", ["full_b512", "full_b2048", "full32_b128"])
def test_oracle_reproduces_the_stored_sensitivity(name):
    """Recomputed here (same perturbation seeds): every tensor and statistic agrees
    with the stored value within a factor of two (BLAS summation order may differ
    between machines, which moves individual rounding flips)."""
    got = sensitivity.measure(sensitivity.CASES[name])
    ref = _golden()["cases"][name]
    for kind, floor in (("grad", 1e-5), ("stat", 1e-7)):
        for n, r in ref[kind].items():
            v = got[kind][n]
            assert v <= 2 * r + floor and r <= 2 * v + floor, (kind, n, v, r)
