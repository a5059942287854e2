"""The oracle's own sensitivity in its bfloat16-operand mode.

Both sides of a BF16 parity test round the same operands to bfloat16, but the
value being rounded is FP32 on the GPU and FP64 in the oracle.  Wherever the two
values straddle a rounding boundary the rounded operands differ by one bfloat16
unit, and every later rounding decision of that row can follow.  How far a
result moves through such flips is a property of the oracle's arithmetic alone,
so it is measured here on the oracle, with a perturbation shaped like FP32's own
error:

  * every computed operand of a contraction (activations, upstream gradients)
    gets x_i <- x_i + delta s_i rms(row of x), s_i = +-1 drawn per element.  An
    FP32 dot product's error scales with the magnitude of its terms, not with
    its result, so the deviation is absolute at the row's scale (small elements
    take large relative deviations, as in FP32).
  * values that the GPU holds exactly are left alone: elements that are exactly
    representable in FP32 (the squinted images, replayed states and actions,
    the exact zeros of ReLU) and every parameter (both sides round the same FP32
    parameter values, so their bfloat16 copies agree exactly).
  * delta = 2^-22, i.e. 4 FP32 rounding units (2^-24) at the row's RMS: the
    mean absolute deviation of FP32 computations of the encoder and critic
    activations from FP64 is 1.4 to 3.6 units at the same scale
    (fp32_deviation() below, recorded with the table).

The largest relative change over the perturbations, per gradient tensor and per
statistic, is the self-sensitivity that the BF16 tolerances of the GPU tests are
derived from (tests/helpers.py: max(stated bar, SENS_FACTOR x sensitivity)).

Only oracle/, the synthetic input generators and (for the FP32 deviation) torch's
CPU float32 arithmetic are used.
"""
import numpy as np

from oracle import bf16 as obf16
from oracle import layout as olayout
from oracle import ring as oring
from oracle import sac
from paper_2602_21203_amd import configs, synthetic

DELTA = 2.0 ** -22
N_PERTURB = 8
PERTURB_SEED = 7
STAT_NAMES = ("critic_loss", "actor_loss", "alpha_loss", "alpha", "entropy", "mean_q", "mean_target")

# every BF16 update case of the GPU parity tests: config, batch, replay rows, and
# the variant switches (atoms = None keeps the config's atoms)
CASES = {
    "tiny_b32": dict(cfg="tiny", B=32, cap=4096),
    "full_b512": dict(cfg="full", B=512, cap=2048),
    "full_b2048": dict(cfg="full", B=2048, cap=4096),
    "full128_b1024": dict(cfg="full128", B=1024, cap=1024),
    "full32_b128": dict(cfg="full32", B=128, cap=512),
    "state_b512": dict(cfg="state", B=512, cap=2048),
    "odd_b32": dict(cfg="odd", B=32, cap=4096),
    "tiny_b100": dict(cfg="tiny", B=100, cap=4096),
    "tiny_scalar_b32": dict(cfg="tiny", B=32, cap=4096, atoms=1),
    "full_cdq_b512": dict(cfg="full", B=512, cap=2048, cdq=True),
    "full_scalar_cdq_b512": dict(cfg="full", B=512, cap=2048, atoms=1, cdq=True),
    # updates sampling a ring of frames squinted at insertion: 40 then 56 raw
    # transitions (seeds 20, 21) into a 96-row ring, after each insertion
    "ring_tiny_b32_0": dict(cfg="tiny", B=32, cap=96, ring_chunks=(40,)),
    "ring_tiny_b32_1": dict(cfg="tiny", B=32, cap=96, ring_chunks=(40, 56)),
}


def case_dims(case):
    cfg = dict(configs.CONFIGS[case["cfg"]])
    if case.get("atoms") is not None:
        cfg["atoms"] = case["atoms"]
    return cfg, olayout.dims(**cfg)


def case_params(case):
    _, d = case_dims(case)
    tab = [(n, o, s) for n, (o, s) in olayout.offsets(d)[0].items()]
    return synthetic.init_params(tab, seed=1)


def ring_batch(cfg, n, seed):
    """n raw transitions for a ring insertion (numpy), as the ring tests draw them."""
    rep = synthetic.replay(n, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=seed,
                           done_rate=0.2)
    rep.pop("size")
    return {k: v.numpy() for k, v in rep.items()}


def case_replay(case):
    cfg, _ = case_dims(case)
    if "ring_chunks" in case:
        r = oring.Ring(case["cap"], cfg["H"] // cfg["k"], cfg["C"], cfg["proprio"], cfg["action"])
        for i, n in enumerate(case["ring_chunks"]):
            b = ring_batch(cfg, n, 20 + i)
            r.insert(cfg["k"], *(b[f] for f in oring.FIELDS))
        return r.replay()
    rep = synthetic.replay(case["cap"], cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0)
    return {k: (v.numpy() if hasattr(v, "numpy") else v) for k, v in rep.items()}


def perturbation(rng, delta):
    """x + delta s rms(row), for every element of x not exactly representable in FP32."""
    def f(x):
        if x.ndim == 0 or x.size == 0:
            return x
        axes = tuple(range(1, x.ndim)) if x.ndim > 1 else (0,)
        rms = np.sqrt(np.mean(x * x, axis=axes, keepdims=True))
        computed = x.astype(np.float32).astype(np.float64) != x
        s = rng.choice(np.array([-1.0, 1.0]), size=x.shape)
        return np.where(computed, x + delta * s * rms, x)
    return f


def _run(d, params, rep, case):
    hp = sac.hparams(d, cdq=bool(case.get("cdq", False)))
    st = sac.new_state(d, params)
    o = sac.sac_update(st, rep, d, hp, case["B"], bf=True)
    g = np.zeros(olayout.blocks(d)["total"])
    blk = olayout.blocks(d)
    g[:blk["critic"][1]] = o["g_enc_critic"]
    g[blk["actor"][0]:blk["actor"][1]] = o["g_actor"]
    g[blk["log_alpha"][0]] = o["g_log_alpha"][0]
    return g, o["stats"], o["stat_scale"]


def measure(case, n_perturb=N_PERTURB, delta=DELTA, rep=None):
    """{"grad": {tensor: sens}, "stat": {name: sens}} for one case."""
    _, d = case_dims(case)
    p0 = case_params(case).astype(np.float64)
    rep = case_replay(case) if rep is None else rep
    g0, s0, sc0 = _run(d, p0, rep, case)
    table = olayout.offsets(d)[0]
    grad = {n: 0.0 for n in table}
    stat = {n: 0.0 for n in STAT_NAMES}
    rng = np.random.default_rng(PERTURB_SEED)
    for _ in range(n_perturb):
        obf16.set_computed_perturbation(perturbation(rng, delta))
        try:
            g, st, _ = _run(d, p0, rep, case)
        finally:
            obf16.set_computed_perturbation(None)
        for n, (o, shp) in table.items():
            k = int(np.prod(shp))
            ref = np.linalg.norm(g0[o:o + k])
            e = float(np.linalg.norm(g[o:o + k] - g0[o:o + k]) / max(ref, 1e-30))
            grad[n] = max(grad[n], e)
        for i, n in enumerate(STAT_NAMES):
            scale = max(abs(s0[i]), sc0[i])
            stat[n] = max(stat[n], float(abs(st[i] - s0[i]) / max(scale, 1e-30)))
    return {"grad": grad, "stat": stat}


# act() in the bfloat16 mode: the full network on 300 replayed frames, mean and
# sampled actions (the GPU act() parity case)
ACT_CASE = dict(cfg="full", cap=2048, n=300, request_id=12345678901)


def measure_act(case=ACT_CASE, n_perturb=N_PERTURB, delta=DELTA, rep=None):
    """{"mean": sens, "sample": sens}: relative-norm change of the action array."""
    _, d = case_dims(case)
    p = case_params(case).astype(np.float64)
    rep = case_replay(case) if rep is None else rep
    n = case["n"]
    hp = sac.hparams(d)
    out = {}
    for key, sample in (("mean", False), ("sample", True)):
        a0 = sac.act(p, d, hp, rep["obs"][:n], rep["proprio"][:n], sample, case["request_id"], bf=True)
        rng = np.random.default_rng(PERTURB_SEED)
        worst = 0.0
        for _ in range(n_perturb):
            obf16.set_computed_perturbation(perturbation(rng, delta))
            try:
                a = sac.act(p, d, hp, rep["obs"][:n], rep["proprio"][:n], sample, case["request_id"], bf=True)
            finally:
                obf16.set_computed_perturbation(None)
            worst = max(worst, float(np.linalg.norm(a - a0) / max(np.linalg.norm(a0), 1e-30)))
        out[key] = worst
    return out


def fp32_deviation(case=None, rows=512):
    """Mean absolute deviation of FP32 computations from FP64, in FP32 rounding
    units (2^-24) at each row's RMS, for the encoder's conv activations, the
    critic projection and the first twin's two hidden layers (full network, torch
    CPU float32 against float64 on the same parameters and replayed rows)."""
    import torch
    import torch.nn.functional as F

    from oracle.squint import squint
    case = CASES["full_b512"] if case is None else case
    _, d = case_dims(case)
    P = olayout.view(case_params(case).astype(np.float64), d)
    rep = case_replay(case)
    x = squint(rep["obs"][:rows], d.k)

    def ln(v, g, b):
        mu = v.mean(-1, keepdim=True)
        var = ((v - mu) ** 2).mean(-1, keepdim=True)
        return g * (v - mu) / torch.sqrt(var + 1e-5) + b

    def forward(dt):
        T = lambda a: torch.tensor(np.asarray(a), dtype=dt)
        h, outs = T(x), {}
        for i in range(d.n_conv):
            h = torch.relu(F.conv2d(h, T(P[f"enc.conv{i + 1}.W"]), T(P[f"enc.conv{i + 1}.b"]),
                                    stride=2 if i == 0 else 1))
            outs[f"conv{i + 1}"] = h.reshape(h.shape[0], -1)
        t = torch.tanh(ln(h.reshape(h.shape[0], -1) @ T(P["critic.trunk.W"]).T + T(P["critic.trunk.b"]),
                          T(P["critic.trunk.ln.g"]), T(P["critic.trunk.ln.b"])))
        outs["critic.trunk"] = t
        X = torch.cat([t, T(rep["proprio"][:rows]), T(rep["action"][:rows])], 1)
        for l in ("l1", "l2"):
            X = torch.relu(ln(X @ T(P[f"q1.{l}.W"]).T + T(P[f"q1.{l}.b"]), T(P[f"q1.{l}.ln.g"]),
                              T(P[f"q1.{l}.ln.b"])))
            outs[f"q1.{l}"] = X
        return outs

    o64, o32 = forward(torch.float64), forward(torch.float32)
    out = {}
    for k in o64:
        a, b = o64[k].numpy(), o32[k].double().numpy()
        rms = np.sqrt(np.mean(a * a, axis=1, keepdims=True))
        out[k] = float(np.mean(np.abs(a - b) / np.maximum(rms, 1e-30)) / 2.0 ** -24)
    return out


# the encoder op parity case (encoder_fwd / encoder_bwd alone): n random frames
# squinted, upstream gradient N(0, 1) (the GPU test's recipe: op_batch below)
ENC_OP_CASES = {"tiny_n37": ("tiny", 37), "full_n77": ("full", 77), "full32_n45": ("full32", 45)}


def op_batch(cfg, n, seed=0):
    """Inputs of the op parity tests: squinted random frames, proprio, actions."""
    from oracle import squint
    rng = np.random.default_rng(seed)
    d = olayout.dims(**cfg)
    x = squint.squint(rng.integers(0, 256, size=(n, cfg["H"], cfg["W"], cfg["C"]), dtype=np.uint8), cfg["k"])
    s = rng.normal(size=(n, cfg["proprio"]))
    a = rng.uniform(-1, 1, size=(n, cfg["action"]))
    return d, x, s, a


def measure_enc_op(name, n, n_perturb=N_PERTURB, delta=DELTA):
    """{"feat": sens, tensor: sens, ...} of the encoder alone in the bfloat16 mode."""
    from oracle import nets
    cfg = dict(configs.CONFIGS[name])
    d, x, _, _ = op_batch(cfg, n)
    tab = [(t, o, sh) for t, (o, sh) in olayout.offsets(d)[0].items()]
    P = olayout.view(synthetic.init_params(tab, seed=1).astype(np.float64), d)
    xf = x.astype(np.float32).astype(np.float64)
    f0, ec = nets.encoder_fwd(P, xf, d.n_conv, True)
    dfeat = np.random.default_rng(1).normal(size=f0.shape)
    g0 = nets.encoder_bwd(P, ec, dfeat, d.n_conv, True)
    out = {"feat": 0.0}
    out.update({t: 0.0 for t in g0})
    rng = np.random.default_rng(PERTURB_SEED)
    for _ in range(n_perturb):
        obf16.set_computed_perturbation(perturbation(rng, delta))
        try:
            f1, ec1 = nets.encoder_fwd(P, xf, d.n_conv, True)
            g1 = nets.encoder_bwd(P, ec1, dfeat, d.n_conv, True)
        finally:
            obf16.set_computed_perturbation(None)
        out["feat"] = max(out["feat"], float(np.linalg.norm(f1 - f0) / np.linalg.norm(f0)))
        for t in g0:
            out[t] = max(out[t], float(np.linalg.norm(g1[t] - g0[t]) / max(np.linalg.norm(g0[t]), 1e-30)))
    return out
