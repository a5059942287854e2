"""Writes bf16_sensitivity.json: the oracle's own bfloat16-mode sensitivity
(tests/sensitivity.py) for every BF16 update case of the GPU parity tests.

Calls only oracle/ and the synthetic input generators.  Run from the repository
root:  python -m tests.golden.make_bf16_sensitivity   (about five minutes)
"""
import json
import os
import sys
import time

from tests import sensitivity

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bf16_sensitivity.json")


def main(names=None):
    out = {"delta": sensitivity.DELTA, "n_perturb": sensitivity.N_PERTURB,
           "perturb_seed": sensitivity.PERTURB_SEED, "cases": {}}
    if os.path.exists(OUT):
        with open(OUT) as f:
            old = json.load(f)
        for k in ("cases", "act", "scaling", "fp32_deviation", "enc_ops"):
            if k in old:
                out[k] = old[k]
    for name, case in sensitivity.CASES.items():
        if names and name not in names:
            continue
        t = time.time()
        out["cases"][name] = dict(case, **sensitivity.measure(case))
        g = out["cases"][name]["grad"]
        worst = max(g, key=g.get)
        print(f"{name}: worst gradient {worst} {g[worst]:.2e}, "
              f"stats max {max(out['cases'][name]['stat'].values()):.2e} ({time.time() - t:.0f} s)", flush=True)
    if not names or "ops" in names:
        out["enc_ops"] = {k: sensitivity.measure_enc_op(*v) for k, v in sensitivity.ENC_OP_CASES.items()}
        print("encoder ops:", out["enc_ops"], flush=True)
    if not names or "fp32_deviation" in names:
        out["fp32_deviation"] = sensitivity.fp32_deviation()
        print("fp32 deviation (units at row RMS):", out["fp32_deviation"], flush=True)
    if not names or "act" in names:
        out["act"] = dict(sensitivity.ACT_CASE, **sensitivity.measure_act())
        print("act:", out["act"], flush=True)
    if not names or "scaling" in names:
        # how the sensitivity grows with the size of the perturbation (full, B = 512)
        case = sensitivity.CASES["full_b512"]
        rep = sensitivity.case_replay(case)
        out["scaling"] = {}
        for e in (24, 22, 20):
            r = sensitivity.measure(case, n_perturb=4, delta=2.0 ** -e, rep=rep)
            out["scaling"][f"2^-{e}"] = {"max_grad": max(r["grad"].values()), "max_stat": max(r["stat"].values()),
                                         "median_grad": float(sorted(r["grad"].values())[len(r["grad"]) // 2])}
            print(f"delta 2^-{e}:", out["scaling"][f"2^-{e}"], flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
