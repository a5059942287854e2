"""GPU parity of the individual entry points against the oracle (C ABI calls)."""
import math

import numpy as np
import pytest
import torch

from oracle import bf16 as obf16
from oracle import layout as olayout
from oracle import nets, philox, sac, squint
from paper_2602_21203_amd import synthetic
from tests import helpers as H
from tests import sensitivity

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_21203_amd import api
    from paper_2602_21203_amd._lib import SQ_BF16, SQ_F32, make_hparams


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.asarray(x), dtype=dtype).cuda().contiguous()


@pytest.mark.parametrize("seed,update,size,n", [(2, 0, 65536, 512), (2, 7, 4096, 4096), (123456789012, 3, 1, 33),
                                                (2, 1, 65537, 1000), (5, 2 ** 31, 2 ** 31 - 1, 257)])
def test_indices_bit_exact(seed, update, size, n):
    print(f"indices seed={seed} update={update} size={size} n={n}", flush=True)
    got = api.sample_indices(seed, update, size, n).cpu().numpy()
    np.testing.assert_array_equal(got, philox.sample_indices(seed, update, size, n))


def test_indices_empty():
    assert api.sample_indices(2, 0, 10, 0).numel() == 0


@pytest.mark.parametrize("stream_id", [1, 2])
def test_gaussian_close_to_fp64(stream_id):
    n = 100003
    got = api.gaussian(2, 9, stream_id, n).cpu().numpy().astype(np.float64)
    ref = philox.gaussian(2, 9, stream_id, n)
    # same uniforms bit for bit; only FP32 log / sqrt / cos rounding differs
    assert np.abs(got - ref).max() < 2e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("name", ["tiny", "full", "full128", "full32"])
def test_squint_bit_exact(name):
    cfg = H.cfg(name)
    print(f"squint {name}", flush=True)
    frames = synthetic.frames(37, cfg["H"], cfg["W"], cfg["C"], seed=4)
    fd = frames.cuda()
    idx = torch.tensor([36, 0, 5, 5, 17, 3, 36], dtype=torch.int32, device="cuda")
    out = api.squint_downsample(cfg, fd, idx)
    want = squint.squint_f32(frames.numpy()[idx.cpu().numpy()], cfg["k"])
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    # no index: rows 0..n-1, ragged count
    out2 = api.squint_downsample(cfg, fd, None, n=37)
    np.testing.assert_array_equal(out2.cpu().numpy(), squint.squint_f32(frames.numpy(), cfg["k"]))
    # bfloat16 output = nearest-even rounding of the FP32 value
    ob = api.squint_downsample(cfg, fd, idx, prec=SQ_BF16)
    wb = torch.tensor(want).to(torch.bfloat16)
    assert torch.equal(ob.cpu(), wb)


def _rand_batch(cfg, n, seed=0):
    return sensitivity.op_batch(cfg, n, seed)


def _tensor_errs(got, ref, tab, base):
    out = {}
    for name, (o, sh) in tab.items():
        k = math.prod(sh)
        if o - base < 0 or o - base + k > len(got):
            continue
        out[name] = H.rel_norm(got[o - base:o - base + k], ref[o - base:o - base + k])
    return out


@pytest.mark.parametrize("name,n,prec", [("tiny", 37, 0), ("full", 77, 0), ("tiny", 37, 1), ("full", 77, 1),
                                         ("full32", 45, 0), ("full32", 45, 1)])
def test_encoder_critic_actor_ops_vs_oracle(name, n, prec):
    print(f"ops {name} n={n} prec={prec}", flush=True)
    cfg = H.cfg(name)
    bf = prec == 1
    d, x, s, a = _rand_batch(cfg, n)
    p64 = H.params(name).astype(np.float64)
    P = olayout.view(p64, d)
    tab, _ = olayout.offsets(d)
    blk = olayout.blocks(d)
    p = dev(p64)
    fwd_tol = 1e-5 if not bf else 1e-3
    # both sides get the same FP32 image
    xf = x.astype(np.float32)
    feat_ref, ec = nets.encoder_fwd(P, xf.astype(np.float64), d.n_conv, bf)
    feat, ws = api.encoder_fwd(cfg, prec, p[:blk["enc"][1]], dev(xf))
    # the bfloat16 encoder's tolerances follow the oracle's own sensitivity of this
    # case (tests/sensitivity.py): on 32 x 32 inputs its gradients are chaotic at 5e-3
    ecase = f"{name}_n{n}"
    tol = (lambda what: H.bf16_enc_op_tol(ecase, what)) if bf else (lambda what: 1e-3)
    e = H.rel_norm(feat.cpu().numpy(), feat_ref)
    print(f"  feat err {e:.2e} tol {min(fwd_tol, tol('feat')) if not bf else max(fwd_tol, tol('feat')):.1e}")
    assert e < (fwd_tol if not bf else max(fwd_tol, tol("feat")))
    rng = np.random.default_rng(1)
    dfeat = rng.normal(size=feat_ref.shape)
    g_ref = nets.encoder_bwd(P, ec, dfeat, d.n_conv, bf)
    g = api.encoder_bwd(cfg, prec, p[:blk["enc"][1]], ws, dev(dfeat), blk["enc"][1]).cpu().numpy()
    for nm, gr in g_ref.items():
        o, sh = tab[nm]
        e = H.rel_norm(g[o:o + gr.size], gr.ravel())
        print(f"  {nm} err {e:.2e} tol {tol(nm):.1e}")
        assert e < tol(nm), nm
    # critic (online parameters, FP64 features so both sides see the same input)
    featq = feat_ref.astype(np.float32).astype(np.float64)
    logits_ref, cc = nets.critic_fwd(P, featq, s, a, bf)
    c0, c1 = blk["critic"]
    logits, cws = api.critic_fwd(cfg, prec, p[c0:c1], dev(featq), dev(s), dev(a))
    assert H.rel_norm(logits.cpu().numpy(), logits_ref) < fwd_tol
    dl = rng.normal(size=logits_ref.shape) * 0.1
    gc_ref, df_ref, da_ref = nets.critic_bwd(P, cc, dl, bf)
    dp, df, da = api.critic_bwd(cfg, prec, p[c0:c1], cws, dev(dl))
    dp = dp.cpu().numpy()
    for nm, gr in gc_ref.items():
        o, sh = tab[nm]
        assert H.rel_norm(dp[o - c0:o - c0 + gr.size], gr.ravel()) < 1e-3, nm
    assert H.rel_norm(df.cpu().numpy(), df_ref) < 1e-3
    assert H.rel_norm(da.cpu().numpy(), da_ref) < 1e-3
    # action-only backward
    _, _, da2 = api.critic_bwd(cfg, prec, p[c0:c1], cws, dev(dl), want_params=False, want_feat=False)
    assert H.rel_norm(da2.cpu().numpy(), da_ref) < 1e-3
    # actor
    hp = make_hparams(cfg["action"], prec=prec)
    eps = rng.normal(size=(n, cfg["action"]))
    a0, a1 = blk["actor"]
    act_ref, lp_ref, acache = nets.actor_fwd(P, featq, s, eps, -5.0, 2.0, bf)
    act, lp, aws = api.actor_fwd(cfg, prec, hp, p[a0:a1], dev(featq), dev(s), dev(eps))
    assert np.abs(act.cpu().numpy() - act_ref).max() < 10 * fwd_tol
    assert H.rel_norm(lp.cpu().numpy(), lp_ref) < fwd_tol
    dact = rng.normal(size=act_ref.shape)
    dlp = rng.normal(size=n)
    ga_ref = nets.actor_bwd(P, acache, dact, dlp, bf)
    ga = api.actor_bwd(cfg, prec, hp, p[a0:a1], aws, dev(dact), dev(dlp)).cpu().numpy()
    for nm, gr in ga_ref.items():
        o, sh = tab[nm]
        assert H.rel_norm(ga[o - a0:o - a0 + gr.size], gr.ravel()) < 1e-3, nm
    # deterministic mean action
    am, _, _ = api.actor_fwd(cfg, prec, hp, p[a0:a1], dev(featq), dev(s), None)
    am_ref, _, _ = nets.actor_fwd(P, featq, s, None, -5.0, 2.0, bf)
    assert np.abs(am.cpu().numpy() - am_ref).max() < 10 * fwd_tol


@pytest.mark.parametrize("N,lo,hi,n", [(51, -10.0, 10.0, 5), (101, -20.0, 20.0, 333), (3, -1.0, 1.0, 4)])
def test_c51_projection_vs_oracle_and_invariants(N, lo, hi, n):
    cfg = dict(H.cfg("full"), atoms=N, v_min=lo, v_max=hi)
    rng = np.random.default_rng(N)
    p = nets.softmax(rng.normal(size=(n, N)) * 2).astype(np.float32)
    r = rng.uniform(-3 * hi / 10, 3 * hi / 10, n).astype(np.float32)
    done = (rng.uniform(size=n) < 0.3).astype(np.uint8)
    bonus = (rng.normal(size=n) * 2).astype(np.float32)
    m = api.c51_project(cfg, dev(p), dev(r), dev(done, torch.uint8), dev(bonus), 0.99).cpu().numpy()
    ref = nets.c51_project(p.astype(np.float64), r.astype(np.float64), done.astype(np.float64), 0.99,
                           bonus.astype(np.float64), lo, hi)
    assert np.abs(m - ref).max() < 1e-5
    assert m.min() >= 0
    np.testing.assert_allclose(m.sum(1), 1.0, atol=2e-6)
    # identity projection at reward 0, gamma 1, not done, no bonus: exact in real
    # arithmetic; in FP32 each atom position b_j = (z_j - v_min) / dz carries the
    # rounding of z_j, about ulp(max|v|) / dz, which moves that much of p_j
    mi = api.c51_project(cfg, dev(p), dev(np.zeros(n)), dev(np.zeros(n), torch.uint8), None, 1.0).cpu().numpy()
    dz = (hi - lo) / (N - 1)
    bound = 4 * np.spacing(np.float32(max(abs(lo), abs(hi)))) / dz
    assert np.abs(mi - p).max() <= bound * p.max() + 1e-7


def test_adam_step_vs_oracle_with_ema_and_shadow():
    rng = np.random.default_rng(3)
    n = 100_003
    p0, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m0, v0 = (rng.normal(size=n) * 0.01).astype(np.float32), np.abs(rng.normal(size=n) * 0.01).astype(np.float32)
    tgt0 = rng.normal(size=n - 1000).astype(np.float32)
    hp = make_hparams(6)
    p, m, v, tgt = dev(p0), dev(m0), dev(v0), dev(tgt0)
    shadow = torch.empty(n, dtype=torch.int16, device="cuda")
    step = torch.tensor([4], dtype=torch.int32, device="cuda")
    api.adam_step(p, dev(g), m, v, hp, step, p_bf16=shadow, ema_target=tgt, ema_begin=1000)
    P, M, V = p0.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64)
    ohp = sac.hparams(olayout.dims(**H.cfg("tiny")))
    sac.adam(P, g.astype(np.float64), M, V, 5, ohp)
    # beta1 = 0.9 and 1 - beta1 are inexact in FP32 (relative 3e-8 / 2.4e-7)
    assert np.abs(p.cpu().numpy() - P).max() < 1e-6
    assert np.abs(m.cpu().numpy() - M).max() < 1e-6
    assert np.abs(v.cpu().numpy() - V).max() < 1e-6
    T = tgt0.astype(np.float64)
    sac.ema(T, P[1000:], 0.995)
    assert np.abs(tgt.cpu().numpy() - T).max() < 1e-6
    assert torch.equal(shadow.view(torch.bfloat16).cpu(), p.cpu().to(torch.bfloat16))
    assert int(step.item()) == 5            # advanced on the device after the step
    # a second step reads t = 6 from the advanced counter
    api.adam_step(p, dev(g), m, v, hp, step)
    sac.adam(P, g.astype(np.float64), M, V, 6, ohp)
    assert np.abs(p.cpu().numpy() - P).max() < 2e-6
    assert int(step.item()) == 6
