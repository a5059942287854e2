"""Pins of the oracle's update variants (the paper's critic ablations, Sec. IV
Critic Design Choices): the clipped double-Q target and the scalar critic with
the squared Bellman error of Eqs. (1)-(2)."""
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
    return torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=grad)


def _setup(cfg, B, cap=128, atoms=None, seed=0, support=None, **hpkw):
    c = dict(getattr(layout, cfg))
    if atoms is not None:
        c["atoms"] = atoms
    if support is not None:
        c["v_min"], c["v_max"] = -support, support
    d = layout.dims(**c)
    cpu = synthetic.replay(cap, d.H, d.W, d.C, d.proprio, d.action, seed=seed)
    rep = {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    tab = [(n, o, s) for n, (o, s) in layout.offsets(d)[0].items()]
    p = synthetic.init_params(tab, seed=1).astype(np.float64)
    return d, rep, sac.new_state(d, p), sac.hparams(d, **hpkw)


def _twins_equal(d, st):
    """Make the target's second twin a copy of the first."""
    tab = layout.offsets(d)[0]
    base = layout.blocks(d)["critic"][0]
    for name, (o, sh) in tab.items():
        if name.startswith("q2."):
            o1, _ = tab["q1." + name[3:]]
            n = math.prod(sh)
            st.target[o - base:o - base + n] = st.target[o1 - base:o1 - base + n]


@pytest.mark.parametrize("atoms", [None, 1])
def test_cdq_equals_average_when_target_twins_agree(atoms):
    d, rep, st, hp = _setup("TINY", 16, atoms=atoms)
    _twins_equal(d, st)
    a = sac.sac_update(sac.copy_state(st), rep, d, hp, 16)
    b = sac.sac_update(sac.copy_state(st), rep, d, sac.hparams(d, cdq=True), 16)
    np.testing.assert_array_equal(a["m"], b["m"])
    np.testing.assert_array_equal(a["stats"], b["stats"])


def test_cdq_target_mean_is_the_smaller_twin_where_nothing_clips():
    """The projection keeps the mean of the shifted support when no atom clips, so
    per row the CDQ target's mean is r + g(1-d)(min_i E_i + bonus), never above the
    averaged target's mean; and rows pick the smaller expectation."""
    # a wide support and a short horizon, so that no shifted atom clips
    d, rep, st, hp = _setup("TINY", 32, support=100.0, gamma=0.5)
    avg = sac.sac_update(sac.copy_state(st), rep, d, hp, 32)
    cdq = sac.sac_update(sac.copy_state(st), rep, d, sac.hparams(d, cdq=True, gamma=0.5), 32)
    z = nets.atoms(d.atoms, d.v_min, d.v_max)
    E = nets.softmax(cdq["logits_bar"]) @ z                    # [2, B]
    r = rep["reward"][cdq["idx"]].astype(np.float64)
    dn = rep["done"][cdq["idx"]].astype(np.float64)
    alpha = math.exp(st.params[layout.blocks(d)["log_alpha"][0]])
    bonus = -alpha * cdq["logp_next"]
    shift = r[:, None] + hp.gamma * (1 - dn[:, None]) * (z[None] + bonus[:, None])
    inside = np.all((shift >= d.v_min) & (shift <= d.v_max), axis=1)
    assert inside.sum() == 32
    want = r + hp.gamma * (1 - dn) * (np.minimum(E[0], E[1]) + bonus)
    np.testing.assert_allclose(cdq["tgt"][inside], want[inside], rtol=1e-12, atol=1e-12)
    assert np.all(cdq["tgt"][inside] <= avg["tgt"][inside] + 1e-12)
    assert np.any(E[1] < E[0]) and np.any(E[0] < E[1])         # both twins get chosen somewhere


@pytest.mark.parametrize("cdq", [False, True])
def test_scalar_target_special_cases(cdq):
    """gamma = 0 leaves y = r; terminal rows give y = r at any gamma."""
    d, rep, st, hp = _setup("TINY", 16, atoms=1, cdq=cdq, gamma=0.0)
    out = sac.sac_update(sac.copy_state(st), rep, d, hp, 16)
    np.testing.assert_array_equal(out["tgt"], rep["reward"][out["idx"]].astype(np.float64))
    rep2 = dict(rep, done=np.ones_like(rep["done"]))
    out = sac.sac_update(sac.copy_state(st), rep2, d, sac.hparams(d, cdq=cdq), 16)
    np.testing.assert_array_equal(out["tgt"], rep["reward"][out["idx"]].astype(np.float64))


def _torch_scalar_grads(d, rep, st, hp, B, out):
    """Gradients of one scalar-critic update from torch autograd."""
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
    alpha = P["log_alpha"][0].detach().exp()
    with torch.no_grad():
        a_n, lp_n = torch_ref.actor(P, f_n, s2, eps_n, hp.log_std_min, hp.log_std_max)
        base = layout.blocks(d)["critic"][0]
        Tt = torch_ref.views(T(st.target), {k: (o - base, sh) for k, (o, sh) in tab.items()
                                            if k.startswith(("critic.", "q1.", "q2."))})
        qb = torch_ref.critic(Tt, f_n, s2, a_n)[..., 0]
        qn = torch.minimum(qb[0], qb[1]) if hp.cdq else qb.mean(0)
        y = r + hp.gamma * (1 - done) * (qn - alpha * lp_n)
    q = torch_ref.critic(P, f_t, s, a)[..., 0]
    loss_c = ((q - y[None]) ** 2).mean(1).sum()
    loss_c.backward()
    g_ec = pt.grad.numpy()[: layout.blocks(d)["critic"][1]].copy()
    pn = T(out["params_after"])
    pa = T(st.params, True)
    a_t, lp_t = torch_ref.actor(torch_ref.views(pa, tab), f_t.detach(), s, eps, hp.log_std_min, hp.log_std_max)
    qa = torch_ref.critic(torch_ref.views(pn, tab), f_t.detach(), s, a_t)[..., 0]
    alpha_new = math.exp(out["params_after"][layout.blocks(d)["log_alpha"][0]])
    loss_pi = (alpha_new * lp_t - 0.5 * (qa[0] + qa[1])).mean()
    loss_pi.backward()
    a0, a1 = layout.blocks(d)["actor"]
    return dict(g_ec=g_ec, g_actor=pa.grad.numpy()[a0:a1], loss_c=float(loss_c.detach()),
                loss_pi=float(loss_pi.detach()), y=y.numpy())


@pytest.mark.parametrize("cfg,B,cdq", [("TINY", 32, False), ("TINY", 32, True), ("FULL", 16, False)])
def test_scalar_critic_update_gradients_vs_autograd(cfg, B, cdq):
    d, rep, st, hp = _setup(cfg, B, atoms=1, cdq=cdq)
    st0 = sac.copy_state(st)
    out = sac.sac_update(st, rep, d, hp, B)
    out["params_after"] = st.params
    ref = _torch_scalar_grads(d, rep, st0, hp, B, out)

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    np.testing.assert_allclose(out["tgt"], ref["y"], rtol=1e-12, atol=1e-12)
    assert rel(out["g_enc_critic"], ref["g_ec"]) < 1e-10
    assert rel(out["g_actor"], ref["g_actor"]) < 1e-10
    assert out["stats"][0] == pytest.approx(ref["loss_c"], rel=1e-12)
    assert out["stats"][1] == pytest.approx(ref["loss_pi"], rel=1e-10, abs=1e-14)


def test_scalar_critic_loss_finite_differences():
    """Central differences of the squared-error critic loss (target frozen)."""
    d, rep, st, hp = _setup("TINY", 16, cap=64, atoms=1)
    B = 16
    st0 = sac.copy_state(st)
    out = sac.sac_update(st, rep, d, hp, B)
    y, idx = out["tgt"], out["idx"]
    x = np.concatenate([squint(rep["obs"][idx], d.k), squint(rep["next_obs"][idx], d.k)])
    s = rep["proprio"][idx].astype(np.float64)
    a = rep["action"][idx].astype(np.float64)

    def loss(p):
        P = layout.view(p, d)
        feat, _ = nets.encoder_fwd(P, x, d.n_conv)
        q, _ = nets.critic_fwd(P, feat[:B], s, a)
        return float(np.sum((q[:, :, 0] - y[None]) ** 2) / B)

    rng = np.random.default_rng(3)
    coords = rng.choice(layout.blocks(d)["critic"][1], 40, replace=False)
    h = 1e-6
    fd = np.array([(loss(st0.params + h * np.eye(1, st0.params.size, c)[0]) -
                    loss(st0.params - h * np.eye(1, st0.params.size, c)[0])) / (2 * h) for c in coords])
    g = out["g_enc_critic"][coords]
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g) + 1e-9


def _torch_state_grads(d, rep, st, hp, B, out):
    """Gradients of one state-based update (no encoder: the states are the
    features) from torch autograd."""
    tab = layout.offsets(d)[0]
    idx = philox.sample_indices(hp.seed, st.u, rep["size"], B)
    eps_n = T(philox.gaussian(hp.seed, st.u, 1, B * d.action).reshape(B, d.action))
    eps = T(philox.gaussian(hp.seed, st.u, 2, B * d.action).reshape(B, d.action))
    g = lambda k: T(rep[k][idx].astype(np.float64))
    s, s2, a, r, done = g("proprio"), g("next_proprio"), g("action"), g("reward"), g("done")
    pt = T(st.params, True)
    P = torch_ref.views(pt, tab)
    alpha = P["log_alpha"][0].detach().exp()
    N = d.atoms
    z = d.v_min + torch.arange(N, dtype=torch.float64) * ((d.v_max - d.v_min) / (N - 1))
    with torch.no_grad():
        a_n, lp_n = torch_ref.actor(P, s2, s2, eps_n, hp.log_std_min, hp.log_std_max)
        base = layout.blocks(d)["critic"][0]
        Tt = torch_ref.views(T(st.target), {k: (o - base, sh) for k, (o, sh) in tab.items()
                                            if k.startswith(("critic.", "q1.", "q2."))})
        lbar = torch_ref.critic(Tt, s2, s2, a_n)
        pbar = 0.5 * (torch.softmax(lbar[0], -1) + torch.softmax(lbar[1], -1))
    m = T(out["m"])
    logits = torch_ref.critic(P, s, s, a)
    loss_c = -(m[None] * F.log_softmax(logits, -1)).sum(-1).mean(1).sum()
    loss_c.backward()
    g_ec = pt.grad.numpy()[: layout.blocks(d)["critic"][1]].copy()
    pn = T(out["params_after"])
    pa = T(st.params, True)
    a_t, lp_t = torch_ref.actor(torch_ref.views(pa, tab), s, s, eps, hp.log_std_min, hp.log_std_max)
    q = torch.softmax(torch_ref.critic(torch_ref.views(pn, tab), s, s, a_t), -1) @ z
    alpha_new = math.exp(out["params_after"][layout.blocks(d)["log_alpha"][0]])
    loss_pi = (alpha_new * lp_t - 0.5 * (q[0] + q[1])).mean()
    loss_pi.backward()
    a0, a1 = layout.blocks(d)["actor"]
    m_ref = nets.c51_project_scatter(pbar.numpy(), r.numpy(), done.numpy(), hp.gamma,
                                     -float(alpha) * lp_n.numpy(), d.v_min, d.v_max)
    return dict(g_ec=g_ec, g_actor=pa.grad.numpy()[a0:a1], loss_c=float(loss_c.detach()),
                loss_pi=float(loss_pi.detach()), m=m_ref)


def test_state_based_update_gradients_vs_autograd():
    """Fig. 7 (left) trains state-based SAC: the same update without the image
    path, the state vector in place of the encoder features."""
    c = dict(layout.TINY, n_conv=0, H=8, W=8, k=1, proprio=40)
    d = layout.dims(**c)
    assert d.flat == 40 and layout.blocks(d)["enc"] == (0, 0)
    cpu = synthetic.replay(128, d.H, d.W, d.C, d.proprio, d.action, seed=0)
    rep = {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    tab = [(n, o, s) for n, (o, s) in layout.offsets(d)[0].items()]
    p = synthetic.init_params(tab, seed=1).astype(np.float64)
    st = sac.new_state(d, p)
    hp = sac.hparams(d)
    st0 = sac.copy_state(st)
    out = sac.sac_update(st, rep, d, hp, 32)
    out["params_after"] = st.params
    ref = _torch_state_grads(d, rep, st0, hp, 32, out)

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    assert rel(out["g_enc_critic"], ref["g_ec"]) < 1e-10
    assert rel(out["g_actor"], ref["g_actor"]) < 1e-10
    assert out["stats"][0] == pytest.approx(ref["loss_c"], rel=1e-12)
    assert out["stats"][1] == pytest.approx(ref["loss_pi"], rel=1e-10, abs=1e-14)
    # the target: torch's twin-averaged softmax projected by the scatter form
    np.testing.assert_allclose(out["m"], ref["m"], atol=1e-12)
