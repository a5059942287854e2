"""Pins of the oracle's layers against torch float64 ops and autograd, and of
the categorical projection / cross entropy against invariants and brute force."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import layout, nets
from oracle.bf16 import round_bf16
from paper_2602_21203_amd import synthetic
from tests import torch_ref

RTOL = 1e-10


def T(x, grad=False):
    return torch.tensor(np.asarray(x), dtype=torch.float64, requires_grad=grad)


def close(a, b, tol=RTOL):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(1.0, float(np.abs(b).max()))
    assert np.abs(a - b).max() <= tol * scale, (np.abs(a - b).max(), scale)


@pytest.mark.parametrize("stride,C,F_,H", [(2, 9, 32, 16), (1, 16, 16, 7), (1, 32, 32, 5)])
def test_conv_fwd_bwd_vs_torch(stride, C, F_, H):
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, C, H, H))
    W = rng.normal(size=(F_, C, 3, 3)) * 0.2
    b = rng.normal(size=F_)
    y = nets.conv_fwd(x, W, b, stride)
    xt, Wt, bt = T(x, True), T(W, True), T(b, True)
    yt = F.conv2d(xt, Wt, bt, stride=stride)
    close(y, yt.detach().numpy())
    dy = rng.normal(size=y.shape)
    yt.backward(T(dy))
    dx, dW, db = nets.conv_bwd(dy, x, W, stride)
    close(dx, xt.grad.numpy())
    close(dW, Wt.grad.numpy())
    close(db, bt.grad.numpy())


@pytest.mark.parametrize("act", ["tanh", "relu"])
def test_dense_ln_act_vs_torch(act):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, 20))
    W = rng.normal(size=(33, 20)) * 0.3
    b, g, be = rng.normal(size=33), 1 + 0.1 * rng.normal(size=33), 0.1 * rng.normal(size=33)
    y, cache = nets.dense_ln_act(x, W, b, g, be, act)
    ts = [T(v, True) for v in (x, W, b, g, be)]
    yt = F.layer_norm(F.linear(ts[0], ts[1], ts[2]), (33,), ts[3], ts[4], eps=1e-5)
    yt = torch.tanh(yt) if act == "tanh" else F.relu(yt)
    close(y, yt.detach().numpy())
    dy = rng.normal(size=y.shape)
    yt.backward(T(dy))
    grads = nets.dense_ln_act_bwd(dy, cache)
    for mine, t in zip(grads, ts):
        close(mine, t.grad.numpy())


def _table(d):
    t, _ = layout.offsets(d)
    return t


def _params(d, seed=1):
    table = [(n, o, s) for n, (o, s) in layout.offsets(d)[0].items()]
    p = synthetic.init_params(table, seed=seed).astype(np.float64)
    # perturb LayerNorm affine so that gain / bias gradients are exercised
    rng = np.random.default_rng(seed + 10)
    for n, (o, s) in layout.offsets(d)[0].items():
        if ".ln." in n:
            p[o:o + math.prod(s)] += 0.1 * rng.normal(size=math.prod(s))
    return p


def _batch(d, n, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.5, 0.5, size=(n, d.C, d.side, d.side))
    s = rng.normal(size=(n, d.proprio))
    a = rng.uniform(-1, 1, size=(n, d.action))
    return x, s, a


def test_layout_counts():
    assert layout.offsets(layout.dims(**layout.FULL))[1] == 1493335
    assert layout.offsets(layout.dims(**layout.TINY))[1] == 90563
    d = layout.dims(**layout.FULL)
    assert d.flat == 288 and d.conv_sides == [7, 5, 3]
    assert layout.blocks(d)["critic"] == (21120, 1010250)


@pytest.mark.parametrize("cfg", ["TINY", "FULL"])
def test_encoder_critic_fwd_bwd_vs_autograd(cfg):
    d = layout.dims(**getattr(layout, cfg))
    p = _params(d)
    P = layout.view(p, d)
    n = 6
    x, s, a = _batch(d, n)
    feat, ec = nets.encoder_fwd(P, x, d.n_conv)
    logits, cc = nets.critic_fwd(P, feat, s, a)
    pt = T(p, True)
    Pt = torch_ref.views(pt, _table(d))
    ft = torch_ref.encoder(Pt, T(x), d.n_conv)
    lt = torch_ref.critic(Pt, ft, T(s), T(a))
    close(feat, ft.detach().numpy())
    close(logits, lt.detach().numpy())
    rng = np.random.default_rng(4)
    dl = rng.normal(size=logits.shape)
    lt.backward(T(dl))
    g, dfeat, _ = nets.critic_bwd(P, cc, dl)
    g.update(nets.encoder_bwd(P, ec, dfeat, d.n_conv))
    want = layout.view(pt.grad.numpy(), d)
    for name, gv in g.items():
        close(gv, want[name])
    # the action gradient on its own (critic params untouched)
    at = T(a, True)
    torch_ref.critic(torch_ref.views(T(p), _table(d)), T(feat), T(s), at).backward(T(dl))
    _, _, da = nets.critic_bwd(P, cc, dl, need_params=False, need_dfeat=False)
    close(da, at.grad.numpy())


@pytest.mark.parametrize("cfg", ["TINY", "FULL"])
def test_actor_fwd_bwd_vs_autograd(cfg):
    d = layout.dims(**getattr(layout, cfg))
    p = _params(d)
    P = layout.view(p, d)
    n = 5
    rng = np.random.default_rng(5)
    f = np.abs(rng.normal(size=(n, d.flat)))
    s = rng.normal(size=(n, d.proprio))
    eps = rng.normal(size=(n, d.action))
    a, logp, cache = nets.actor_fwd(P, f, s, eps, -5.0, 2.0)
    pt = T(p, True)
    at, lpt = torch_ref.actor(torch_ref.views(pt, _table(d)), T(f), T(s), T(eps), -5.0, 2.0)
    close(a, at.detach().numpy())
    close(logp, lpt.detach().numpy(), 1e-9)
    da = rng.normal(size=a.shape)
    dlp = rng.normal(size=n)
    ((at * T(da)).sum() + (lpt * T(dlp)).sum()).backward()
    g = nets.actor_bwd(P, cache, da, dlp)
    want = layout.view(pt.grad.numpy(), d)
    for name, gv in g.items():
        close(gv, want[name], 1e-9)


def test_tanh_gaussian_standard_point():
    """mu = 0, sigma = 1, eps = 0 => log pi = -(A/2) log 2 pi (Jacobian is 1 at u = 0)."""
    d = layout.dims(**layout.TINY)
    p = np.zeros(layout.offsets(d)[1])
    P = layout.view(p, d)
    for n_ in ("actor.trunk.ln.g", "actor.l1.ln.g", "actor.l2.ln.g"):
        P[n_][:] = 1.0
    # log sigma = lo + (hi - lo)(tanh(us) + 1)/2 = 0  <=>  tanh(us) = -1 - 2 lo / (hi - lo)
    lo, hi = -5.0, 2.0
    P["actor.out.b"][d.action:] = np.arctanh(-1 - 2 * lo / (hi - lo))
    a, logp, _ = nets.actor_fwd(P, np.zeros((3, d.flat)), np.zeros((3, d.proprio)),
                                np.zeros((3, d.action)), lo, hi)
    assert np.all(a == 0)
    np.testing.assert_allclose(logp, -0.5 * d.action * np.log(2 * np.pi), rtol=1e-12)


# ---------------------------------------------------------------- C51
def _rand_p(rng, n, N):
    return nets.softmax(rng.normal(size=(n, N)) * 2)


def test_projection_mass_and_nonnegativity():
    rng = np.random.default_rng(6)
    for N, lo, hi in ((51, -10, 10), (101, -20, 20)):
        p = _rand_p(rng, 64, N)
        r = rng.uniform(-3, 3, 64)
        done = (rng.uniform(size=64) < 0.2).astype(float)
        bonus = rng.normal(size=64) * 5
        m = nets.c51_project(p, r, done, 0.99, bonus, lo, hi)
        assert m.min() >= 0
        np.testing.assert_allclose(m.sum(1), 1.0, atol=1e-12)


def test_projection_identity():
    rng = np.random.default_rng(7)
    p = _rand_p(rng, 16, 101)
    m = nets.c51_project(p, np.zeros(16), np.zeros(16), 1.0, np.zeros(16), -20, 20)
    np.testing.assert_allclose(m, p, atol=1e-12)


def test_projection_mean_preservation():
    rng = np.random.default_rng(8)
    N, lo, hi = 101, -20.0, 20.0
    z = nets.atoms(N, lo, hi)
    p = _rand_p(rng, 32, N)
    # keep every shifted atom inside the support: |r| small, gamma < 1, bonus small
    r = rng.uniform(-0.1, 0.1, 32)
    bonus = rng.uniform(-0.1, 0.1, 32)
    m = nets.c51_project(p, r, np.zeros(32), 0.9, bonus, lo, hi)
    want = r + 0.9 * (p @ z + bonus)
    np.testing.assert_allclose(m @ z, want, atol=1e-12)


def test_projection_matches_scatter_form_and_is_linear():
    rng = np.random.default_rng(9)
    N, lo, hi = 51, -10.0, 10.0
    p1, p2 = _rand_p(rng, 12, N), _rand_p(rng, 12, N)
    r = rng.uniform(-15, 15, 12)  # exercises both clamps
    done = (rng.uniform(size=12) < 0.3).astype(float)
    bonus = rng.normal(size=12) * 3
    m1 = nets.c51_project(p1, r, done, 0.99, bonus, lo, hi)
    np.testing.assert_allclose(m1, nets.c51_project_scatter(p1, r, done, 0.99, bonus, lo, hi), atol=1e-14)
    m2 = nets.c51_project(p2, r, done, 0.99, bonus, lo, hi)
    m12 = nets.c51_project(0.3 * p1 + 0.7 * p2, r, done, 0.99, bonus, lo, hi)
    np.testing.assert_allclose(m12, 0.3 * m1 + 0.7 * m2, atol=1e-14)


def test_projection_terminal_two_hot():
    N, lo, hi = 51, -10.0, 10.0
    p = _rand_p(np.random.default_rng(10), 4, N)
    r = np.array([0.3, -12.0, 10.5, 2.0])
    m = nets.c51_project(p, r, np.ones(4), 0.99, np.array([1.0, 2.0, 3.0, 4.0]), lo, hi)
    dz = (hi - lo) / (N - 1)
    for i in range(4):
        b = (min(max(r[i], lo), hi) - lo) / dz
        want = np.zeros(N)
        l_ = int(np.floor(b))
        if l_ == b:
            want[l_] = 1
        else:
            want[l_], want[l_ + 1] = l_ + 1 - b, b - l_
        np.testing.assert_allclose(m[i], want, atol=1e-12)


def test_projection_brute_force_three_atoms():
    """N = 3 on [-1, 1] (dz = 1), p = (0.2, 0.3, 0.5), hand-enumerated positions."""
    p = np.array([[0.2, 0.3, 0.5]])
    # r = 0.5, gamma = 0.5, bonus = 0: Tz = (0, 0.5, 1) -> b = (1, 1.5, 2)
    m = nets.c51_project(p, np.array([0.5]), np.zeros(1), 0.5, np.zeros(1), -1.0, 1.0)
    np.testing.assert_allclose(m, [[0.0, 0.2 + 0.15, 0.15 + 0.5]], atol=1e-15)
    # r = -3: everything clamps to the lowest atom
    m = nets.c51_project(p, np.array([-3.0]), np.zeros(1), 1.0, np.zeros(1), -1.0, 1.0)
    np.testing.assert_allclose(m, [[1.0, 0.0, 0.0]], atol=1e-15)
    # r = 2, gamma = 1: Tz = (1, 2, 3) -> all clamp to the top atom
    m = nets.c51_project(p, np.array([2.0]), np.zeros(1), 1.0, np.zeros(1), -1.0, 1.0)
    np.testing.assert_allclose(m, [[0.0, 0.0, 1.0]], atol=1e-15)
    # bonus = 0.25, gamma = 1, r = 0: Tz = (-0.75, 0.25, 1.25) -> b = (0.25, 1.25, 2)
    m = nets.c51_project(p, np.zeros(1), np.zeros(1), 1.0, np.array([0.25]), -1.0, 1.0)
    np.testing.assert_allclose(m, [[0.15, 0.05 + 0.225, 0.075 + 0.5]], atol=1e-15)


def test_cross_entropy_and_expected_q():
    rng = np.random.default_rng(12)
    logits = rng.normal(size=(2, 8, 51))
    m = nets.softmax(logits[0])
    loss, dl = nets.cross_entropy(logits, m)
    np.testing.assert_allclose(dl[0], 0.0, atol=1e-15)
    ent = -np.sum(m * np.log(m), axis=1).mean()
    ce2 = -np.sum(m * F.log_softmax(T(logits[1]), -1).numpy(), axis=1).mean()
    assert loss == pytest.approx(ent + ce2, rel=1e-12)
    lt = T(logits, True)
    (-(T(m)[None] * F.log_softmax(lt, -1)).sum(-1).mean(1).sum()).backward()
    close(dl, lt.grad.numpy(), 1e-12)
    z = nets.atoms(51, -10, 10)
    onehot = np.full((1, 51), -1e3)
    onehot[0, 17] = 0.0
    q, _ = nets.expected_q(onehot, z)
    assert q[0] == pytest.approx(z[17], abs=1e-12)
    lt = T(logits, True)
    (torch.softmax(lt, -1) @ T(z)).sum().backward()
    _, dq = nets.expected_q(logits, z)
    close(dq, lt.grad.numpy(), 1e-12)


def test_bf16_rounding_matches_torch_cast():
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32),
                        (rng.normal(size=2000) * 1e-30).astype(np.float32),
                        (rng.normal(size=2000) * 1e30).astype(np.float32)])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x.astype(np.float64)), want)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 -> 1
    assert round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_bf16_operand_mode_forward_vs_torch_casts():
    d = layout.dims(**layout.TINY)
    p = _params(d)
    P = layout.view(p, d)
    rng = np.random.default_rng(14)
    f = np.abs(rng.normal(size=(9, d.flat)))
    s = rng.normal(size=(9, d.proprio))
    a = rng.uniform(-1, 1, size=(9, d.action))
    logits, _ = nets.critic_fwd(P, f, s, a, bf=True)
    want = torch_ref.critic_bf16_fwd(torch_ref.views(T(p), _table(d)), T(f), T(s), T(a)).numpy()
    # torch rounds FP64 -> FP32 -> BF16 (two roundings) where the oracle rounds once;
    # they agree except on exact double-rounding ties, which random data does not hit
    close(logits, want, 1e-12)
    full, _ = nets.critic_fwd(P, f, s, a, bf=False)
    assert np.abs(full - logits).max() > 1e-5   # the mode changes the result
