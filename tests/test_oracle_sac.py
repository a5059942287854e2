"""Pins of the oracle's full update: optimiser closed forms, the temperature
direction, and every gradient of one update against torch autograd on an
independently stated graph (target recomputed in torch, projection by the
scatter form)."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import layout, nets, philox, sac
from oracle.squint import squint
from paper_2602_21203_amd import synthetic
from tests import torch_ref



def T(x, grad=False):
    return torch.tensor(np.asarray(x), dtype=torch.float64, requires_grad=grad)


def np_replay(d, cap, seed=0):
    rep = synthetic.replay(cap, d.H, d.W, d.C, d.proprio, d.action, seed=seed)
    return {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in rep.items()}


def table(d):
    return [(n, o, s) for n, (o, s) in layout.offsets(d)[0].items()]


def test_adam_first_step_closed_form():
    hp = sac.hparams(layout.dims(**layout.TINY))
    g = np.array([1e-3, -2.0, 5e-9, 0.0, 3.0])
    p, m, v = np.zeros(5), np.zeros(5), np.zeros(5)
    sac.adam(p, g, m, v, 1, hp)
    np.testing.assert_allclose(p, -hp.lr * g / (np.abs(g) + hp.adam_eps), rtol=1e-12, atol=0)


def test_adam_matches_torch_optim_10_steps():
    hp = sac.hparams(layout.dims(**layout.TINY))
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=50)
    gs = rng.normal(size=(10, 50))
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    pt = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=hp.lr, betas=(hp.beta1, hp.beta2), eps=hp.adam_eps)
    for t in range(10):
        sac.adam(p, gs[t], m, v, t + 1, hp)
        pt.grad = torch.tensor(gs[t])
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_ema_closed_form():
    rng = np.random.default_rng(1)
    t0, th = rng.normal(size=20), rng.normal(size=20)
    t = t0.copy()
    for _ in range(37):
        sac.ema(t, th, 0.995)
    np.testing.assert_allclose(t, 0.995 ** 37 * t0 + (1 - 0.995 ** 37) * th, rtol=1e-12)


def _setup(cfg, B, cap=256, seed=0, **hpkw):
    d = layout.dims(**getattr(layout, cfg))
    rep = np_replay(d, cap, seed)
    p = synthetic.init_params(table(d), seed=1).astype(np.float64)
    st = sac.new_state(d, p)
    hp = sac.hparams(d, **hpkw)
    return d, rep, st, hp


def test_temperature_moves_toward_target_entropy():
    d, rep, st, hp = _setup("TINY", 32)
    probe = sac.copy_state(st)
    ent = sac.sac_update(probe, rep, d, hp, 32)["stats"][4]
    for delta, sign in ((+1.0, +1), (-1.0, -1)):
        s2 = sac.copy_state(st)
        hp2 = sac.hparams(d, target_entropy=ent + delta)
        out = sac.sac_update(s2, rep, d, hp2, 32)
        assert out["stats"][4] == pytest.approx(ent)
        alpha1 = out["stats"][3]
        assert np.sign(alpha1 - 1.0) == sign  # log alpha starts at 0


def _torch_update_grads(d, rep, st, hp, B, out):
    """Gradients of one update from torch autograd on an independently stated graph."""
    tab = layout.offsets(d)[0]
    idx = philox.sample_indices(hp.seed, st.u, rep["size"], B)
    eps_n = T(philox.gaussian(hp.seed, st.u, 1, B * d.action).reshape(B, d.action))
    eps = T(philox.gaussian(hp.seed, st.u, 2, B * d.action).reshape(B, d.action))
    g = lambda k: T(rep[k][idx].astype(np.float64))
    s, s2, a, r, done = g("proprio"), g("next_proprio"), g("action"), g("reward"), g("done")
    x = T(np.concatenate([squint(rep["obs"][idx], d.k), squint(rep["next_obs"][idx], d.k)]))
    pt = T(st.params, True)
    P = torch_ref.views(pt, tab)
    feat = torch_ref.encoder(P, x, d.n_conv)
    f_t, f_n = feat[:B], feat[B:]
    log_alpha = P["log_alpha"][0]
    alpha = log_alpha.detach().exp()
    with torch.no_grad():
        a_n, lp_n = torch_ref.actor(P, f_n, s2, eps_n, hp.log_std_min, hp.log_std_max)
        base = layout.blocks(d)["critic"][0]
        Tt = torch_ref.views(T(st.target), {k: (o - base, sh) for k, (o, sh) in tab.items()
                                            if k.startswith(("critic.", "q1.", "q2."))})
        lbar = torch_ref.critic(Tt, f_n, s2, a_n)
        pbar = 0.5 * (torch.softmax(lbar[0], -1) + torch.softmax(lbar[1], -1))
        N = d.atoms
        dz = (d.v_max - d.v_min) / (N - 1)
        z = d.v_min + torch.arange(N, dtype=torch.float64) * dz
        Tz = (r[:, None] + hp.gamma * (1 - done[:, None]) * (z[None] - alpha * lp_n[:, None]))
        bpos = ((Tz.clamp(d.v_min, d.v_max) - d.v_min) / dz)
        lo, hi = bpos.floor().long(), bpos.ceil().long()
        m = torch.zeros(B, N, dtype=torch.float64)
        wl = torch.where(lo == hi, pbar, pbar * (hi - bpos))
        m.scatter_add_(1, lo, wl)
        m.scatter_add_(1, hi, torch.where(lo == hi, torch.zeros_like(pbar), pbar * (bpos - lo)))
    np.testing.assert_allclose(out["m"], m.numpy(), atol=1e-12)
    logits = torch_ref.critic(P, f_t, s, a)
    loss_c = -(m[None] * F.log_softmax(logits, -1)).sum(-1).mean(1).sum()
    loss_c.backward()
    g_ec = pt.grad.numpy()[: layout.blocks(d)["critic"][1]].copy()
    # temperature
    la = T([st.params[layout.blocks(d)["log_alpha"][0]]], True)
    a_t, lp_t = torch_ref.actor(torch_ref.views(T(st.params), tab), f_t.detach(), s, eps,
                                hp.log_std_min, hp.log_std_max)
    (la.exp() * (-lp_t.detach() - hp.target_entropy).mean()).sum().backward()
    # actor against the updated critic (post-step params from the oracle's state)
    pn = T(out["params_after"])
    pa = T(st.params, True)
    Pa = torch_ref.views(pa, tab)
    a_t, lp_t = torch_ref.actor(Pa, f_t.detach(), s, eps, hp.log_std_min, hp.log_std_max)
    lq = torch_ref.critic(torch_ref.views(pn, tab), f_t.detach(), s, a_t)
    q = torch.softmax(lq, -1) @ z
    alpha_new = math.exp(out["params_after"][layout.blocks(d)["log_alpha"][0]])
    loss_pi = (alpha_new * lp_t - 0.5 * (q[0] + q[1])).mean()
    loss_pi.backward()
    a0, a1 = layout.blocks(d)["actor"]
    return dict(g_ec=g_ec, g_la=la.grad.numpy(), g_actor=pa.grad.numpy()[a0:a1],
                loss_c=float(loss_c.detach()), loss_pi=float(loss_pi.detach()))


@pytest.mark.parametrize("cfg,B", [("TINY", 32), ("FULL", 24)])
def test_full_update_gradients_vs_autograd(cfg, B):
    d, rep, st, hp = _setup(cfg, B, cap=128)
    st0 = sac.copy_state(st)
    out = sac.sac_update(st, rep, d, hp, B)
    out["params_after"] = st.params
    ref = _torch_update_grads(d, rep, st0, hp, B, out)

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    assert rel(out["g_enc_critic"], ref["g_ec"]) < 1e-10
    assert rel(out["g_log_alpha"], ref["g_la"]) < 1e-10
    assert rel(out["g_actor"], ref["g_actor"]) < 1e-10
    assert out["stats"][0] == pytest.approx(ref["loss_c"], rel=1e-12)
    assert out["stats"][1] == pytest.approx(ref["loss_pi"], rel=1e-10, abs=1e-14)
    # per-tensor check of every gradient block that is non-trivially routed
    tab = layout.offsets(d)[0]
    for name in ("enc.conv1.W", "critic.trunk.ln.g", "q2.l1.W", "q1.out.b"):
        o, sh = tab[name]
        n = math.prod(sh)
        assert rel(out["g_enc_critic"][o:o + n], ref["g_ec"][o:o + n]) < 1e-10


def test_critic_loss_finite_differences_tiny():
    """Central differences of the critic loss (target frozen) on 40 coordinates."""
    d, rep, st, hp = _setup("TINY", 16, cap=64)
    B = 16
    st0 = sac.copy_state(st)
    out = sac.sac_update(st, rep, d, hp, B)
    m = out["m"]
    idx = out["idx"]
    x = np.concatenate([squint(rep["obs"][idx], d.k), squint(rep["next_obs"][idx], d.k)])
    s = rep["proprio"][idx].astype(np.float64)
    a = rep["action"][idx].astype(np.float64)

    def loss(p):
        P = layout.view(p, d)
        feat, _ = nets.encoder_fwd(P, x, d.n_conv)
        logits, _ = nets.critic_fwd(P, feat[:B], s, a)
        return nets.cross_entropy(logits, m)[0]

    rng = np.random.default_rng(3)
    hi = layout.blocks(d)["critic"][1]
    coords = rng.choice(hi, 40, replace=False)
    h = 1e-6
    fd = []
    for c in coords:
        pp, pm = st0.params.copy(), st0.params.copy()
        pp[c] += h
        pm[c] -= h
        fd.append((loss(pp) - loss(pm)) / (2 * h))
    fd = np.array(fd)
    g = out["g_enc_critic"][coords]
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g) + 1e-9


def test_nan_reward_makes_the_update_non_finite():
    """A NaN reward at a sampled row: the projection's clamp keeps the NaN, so the
    row's target distribution, the critic loss and the mean target are NaN and
    the statistics' non-finite flag is set."""
    d = layout.dims(**layout.TINY)
    rep = np_replay(d, 256)
    hp = sac.hparams(d)
    rows = philox.sample_indices(hp.seed, 0, 256, 16)
    rep["reward"] = rep["reward"].copy()
    rep["reward"][rows[0]] = np.nan
    st = sac.new_state(d, synthetic.init_params(table(d), seed=1))
    o = sac.sac_update(st, rep, d, hp, 16)
    assert np.isnan(o["m"][0]).all() and np.isfinite(o["m"][1:]).all()
    assert o["stats"][7] == 1.0 and np.isnan(o["stats"][0]) and np.isnan(o["stats"][6])
    assert np.isfinite(o["stats"][[2, 3, 4, 5]]).all()


HEAD_MU, HEAD_US = 0.3, -0.4   # the actor head's constant outputs in the closed-form case


def silent_heads_case(d, cap=256, seed=1, terminal=True):
    """Parameters whose twin critic heads (weights and biases, online and hence
    the target copy) are zero and whose actor head has zero weights (every row's
    head output is its bias: mu = HEAD_MU, u_sigma = HEAD_US), and a replay whose
    transitions are all terminal."""
    params = synthetic.init_params(table(d), seed=seed).astype(np.float64)
    offs = layout.offsets(d)[0]
    for n in ("q1.out.W", "q1.out.b", "q2.out.W", "q2.out.b", "actor.out.W"):
        o, shp = offs[n]
        params[o:o + int(np.prod(shp))] = 0.0
    o, _ = offs["actor.out.b"]
    params[o:o + d.action] = HEAD_MU
    params[o + d.action:o + 2 * d.action] = HEAD_US
    rep = np_replay(d, cap)
    rep["done"] = np.ones_like(rep["done"]) if terminal else np.zeros_like(rep["done"])
    return params, rep


def head_logp(d, hp, B, stream):
    """log pi of every row when every head is (HEAD_MU, HEAD_US): the
    tanh-Gaussian density (Eq. (3)) at the policy noise of Philox stream
    `stream` of update 0 (2: the sample at s_t, 1: at s_t+1), written out with
    log(1 - tanh^2 u) taken directly."""
    eps = philox.gaussian(hp.seed, 0, stream, B * d.action).reshape(B, d.action)
    log_sigma = hp.log_std_min + 0.5 * (hp.log_std_max - hp.log_std_min) * (math.tanh(HEAD_US) + 1.0)
    u = HEAD_MU + math.exp(log_sigma) * eps
    return np.sum(-0.5 * eps ** 2 - 0.5 * math.log(2.0 * math.pi) - log_sigma - np.log(1.0 - np.tanh(u) ** 2), axis=1)


def head_closed_form(d, hp, B, alpha):
    """With zero critic heads the critics' expected value is the mean atom for
    every action, so with lr = 0 (the critic still silent after its step) the
    actor loss is alpha mean(log pi) - mean atom and its gradient reaches only
    the actor head's bias: d log pi / d mu = 2 tanh u per dimension, and
    d log pi / d u_sigma = (-1 + 2 tanh(u) sigma eps) (hi - lo)/2 (1 - tanh^2 u_sigma),
    each scaled by alpha / B and summed over the batch."""
    eps = philox.gaussian(hp.seed, 0, 2, B * d.action).reshape(B, d.action)
    lo, hi = hp.log_std_min, hp.log_std_max
    sigma = math.exp(lo + 0.5 * (hi - lo) * (math.tanh(HEAD_US) + 1.0))
    t = np.tanh(HEAD_MU + sigma * eps)
    g_mu = alpha / B * np.sum(2.0 * t, axis=0)
    g_us = alpha / B * np.sum(-1.0 + 2.0 * t * sigma * eps, axis=0) * 0.5 * (hi - lo) * (1.0 - math.tanh(HEAD_US) ** 2)
    return np.concatenate([g_mu, g_us])


def head_entropy(d, hp, B):
    """The update's entropy statistic, -mean log pi of the sample at s_t."""
    return float(-np.mean(head_logp(d, hp, B, 2)))


def silent_heads_closed_form(d, rep, rows, alpha0):
    """What one update must give when every critic logit is zero (uniform softmax
    p = 1/N) and every transition is terminal (the shifted support collapses to
    r, so the projected target is the two-hot of r): critic loss = 2 log N (twin
    cross entropies summed, batch mean); mean Q = mean of the atoms; mean target
    = mean r; head-bias gradient of each twin = 1/N - mean_b two-hot(r_b); every
    other critic and encoder gradient zero (the heads pass nothing back)."""
    N = d.atoms
    z = np.linspace(d.v_min, d.v_max, N)
    r = rep["reward"][rows].astype(np.float64)
    b = (np.clip(r, d.v_min, d.v_max) - d.v_min) / ((d.v_max - d.v_min) / (N - 1))
    two_hot = np.maximum(0.0, 1.0 - np.abs(b[:, None] - np.arange(N)[None, :]))
    return dict(loss=2.0 * math.log(N), mean_q=float(z.mean()), mean_target=float(r.mean()),
                g_bias=1.0 / N - two_hot.mean(axis=0), alpha0=alpha0)


@pytest.mark.parametrize("cfg", ["tiny", "full"])
def test_soft_target_closed_form_with_silent_heads(cfg):
    """Non-terminal transitions with silent critic heads: the averaged target
    softmax is uniform, so the target distribution is the uniform one over the
    shifted, discounted atoms r + gamma (z - alpha log pi'), projected.  With
    gamma = 1/4 no shifted atom leaves the support, so the projection keeps the
    mean: mean target = mean_b (r_b + gamma (mean z - alpha log pi'_b)), with
    log pi' the constant head's density at the noise of the sample at s_t+1
    (Philox stream 1).  The cross entropy of uniform logits is still log N per twin."""
    from paper_2602_21203_amd import configs
    d = layout.dims(**configs.CONFIGS[cfg])
    params, rep = silent_heads_case(d, terminal=False)
    hp = sac.hparams(d, gamma=0.25)
    B = 32
    rows = philox.sample_indices(hp.seed, 0, 256, B)
    alpha0 = float(np.exp(params[layout.blocks(d)["log_alpha"][0]]))
    r = rep["reward"][rows].astype(np.float64)
    z = np.linspace(d.v_min, d.v_max, d.atoms)
    logp_next = head_logp(d, hp, B, 1)
    shifted = r[:, None] + hp.gamma * (z[None, :] - alpha0 * logp_next[:, None])
    assert shifted.min() > d.v_min and shifted.max() < d.v_max   # nothing clips
    o = sac.sac_update(sac.new_state(d, params), rep, d, hp, B)
    s = o["stats"]
    want = float(np.mean(r + hp.gamma * (z.mean() - alpha0 * logp_next)))
    assert abs(s[6] - want) <= 1e-12 * (abs(want) + 1.0)
    assert abs(s[0] - 2.0 * math.log(d.atoms)) <= 1e-12 * s[0]


@pytest.mark.parametrize("cfg", ["tiny", "full"])
def test_whole_update_closed_form_with_silent_heads(cfg):
    """The composition of one whole update on a case with a closed form (see
    silent_heads_closed_form, head_entropy and head_closed_form): the critic
    statistics and gradients, the entropy and the temperature loss
    alpha (entropy - target entropy), and, with lr = 0 so that the critic the
    actor scores against is still silent, the actor loss and gradient."""
    from paper_2602_21203_amd import configs
    d = layout.dims(**configs.CONFIGS[cfg])
    params, rep = silent_heads_case(d)
    hp = sac.hparams(d, lr=0.0)
    B = 32
    offs = layout.offsets(d)[0]
    st = sac.new_state(d, params)
    rows = philox.sample_indices(hp.seed, 0, 256, B)
    cf = silent_heads_closed_form(d, rep, rows, float(np.exp(params[layout.blocks(d)["log_alpha"][0]])))
    o = sac.sac_update(st, rep, d, hp, B)
    s = o["stats"]
    assert abs(s[0] - cf["loss"]) <= 1e-12 * cf["loss"]
    assert abs(s[5] - cf["mean_q"]) <= 1e-12 * (abs(d.v_min) + abs(d.v_max))
    assert abs(s[6] - cf["mean_target"]) <= 1e-12
    ent = head_entropy(d, hp, B)
    assert abs(s[4] - ent) <= 1e-12 * abs(ent)
    assert abs(s[2] - cf["alpha0"] * (ent - hp.target_entropy)) <= 1e-12 * abs(s[2]) + 1e-15
    # lr = 0: the actor loss and gradient against the silent critic
    assert s[3] == cf["alpha0"]
    assert abs(s[1] - (-cf["alpha0"] * ent - cf["mean_q"])) <= 1e-12 * abs(cf["alpha0"] * ent)
    ga = o["g_actor"]
    a0 = layout.blocks(d)["actor"][0]
    for n, (off, shp) in offs.items():
        if not n.startswith("actor."):
            continue
        k = int(np.prod(shp))
        if n == "actor.out.b":
            np.testing.assert_allclose(ga[off - a0:off - a0 + k], head_closed_form(d, hp, B, cf["alpha0"]), rtol=1e-12,
                                       atol=1e-15)
        elif n != "actor.out.W":
            assert np.all(ga[off - a0:off - a0 + k] == 0.0), n
    g = o["g_enc_critic"]
    for n, (off, shp) in offs.items():
        if off >= layout.blocks(d)["critic"][1]:
            continue
        k = int(np.prod(shp))
        if n in ("q1.out.b", "q2.out.b"):
            np.testing.assert_allclose(g[off:off + k], cf["g_bias"], rtol=0, atol=1e-14)
        elif n not in ("q1.out.W", "q2.out.W"):
            assert np.all(g[off:off + k] == 0.0), n
