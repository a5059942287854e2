"""GPU parity of the fused SAC update (sac_update through the C ABI) against
the oracle, plus graph / eager / run-to-run bitwise identity."""
import math

import numpy as np
import pytest
import torch

from oracle import layout as olayout
from oracle import philox, sac
from paper_2602_21203_amd import synthetic
from tests import helpers as H

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_21203_amd import api

_REPLAYS = {}


def replay(name, cap):
    key = (name, cap)
    if key not in _REPLAYS:
        cfg = H.cfg(name)
        cpu = synthetic.replay(cap, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0)
        gpu = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in cpu.items()}
        _REPLAYS[key] = (H.np_replay(cpu), gpu)
    return _REPLAYS[key]


STAT_NAMES = ("critic_loss", "actor_loss", "alpha_loss", "alpha", "entropy", "mean_q", "mean_target")


def report_grads(g, out, d, case):
    """Print every gradient tensor's relative error (and its BF16 tolerance)."""
    blk = olayout.blocks(d)
    ref = np.zeros(blk["total"])
    ref[:blk["critic"][1]] = out["g_enc_critic"]
    ref[blk["actor"][0]:blk["actor"][1]] = out["g_actor"]
    ref[blk["log_alpha"][0]] = out["g_log_alpha"][0]
    for n, (o, shp) in olayout.offsets(d)[0].items():
        k = int(np.prod(shp))
        tol = H.GRAD_RTOL if case is None else H.bf16_grad_tol(case, n)
        print(f"  PARITY {case or 'fp32'} {n} err {H.rel_norm(g[o:o + k], ref[o:o + k]):.3e} tol {tol:.2e}")


def gpu_run(name, B, cap, prec, n_updates, graph=True, policy_freq=1, chunks=1):
    cfg = H.cfg(name)
    _, rep = replay(name, cap)
    ag = api.Agent(cfg, H.params(name), B, prec=prec, policy_freq=policy_freq)
    stats = []
    for _ in range(chunks):
        stats.append(ag.sac_update(rep, n_updates, graph=graph))
    torch.cuda.synchronize()
    return ag, torch.cat(stats).cpu().numpy()


def oracle_run(name, B, cap, prec, n_updates, policy_freq=1):
    d = H.odims(name)
    rep, _ = replay(name, cap)
    hp = sac.hparams(d, policy_freq=policy_freq)
    st = sac.new_state(d, H.params(name).astype(np.float64))
    outs = [sac.sac_update(st, rep, d, hp, B, bf=prec == 1) for _ in range(n_updates)]
    return st, outs


@pytest.mark.parametrize("name,B,cap,prec", [("tiny", 32, 4096, 0), ("full", 512, 2048, 0),
                                             ("tiny", 32, 4096, 1), ("full", 512, 2048, 1),
                                             ("full32", 128, 512, 0), ("full32", 128, 512, 1),
                                             ("state_tiny", 32, 256, 0), ("state", 512, 2048, 0),
                                             ("state", 512, 2048, 1),
                                             # the other benchmarked shapes: batch 2048 in BF16, and the
                                             # UTD-sweep shape (batch 1024, 128x128 frames squinted 8x)
                                             ("full", 2048, 4096, 1), ("full128", 1024, 1024, 1),
                                             # widths off the kernels' tiles (the general-shape paths)
                                             ("odd", 32, 4096, 0), ("odd", 32, 4096, 1)])
def test_one_update_matches_oracle(name, B, cap, prec):
    print(f"update parity {name} B={B} prec={prec}", flush=True)
    case = f"{name}_b{B}" if prec == 1 else None
    ag, stats = gpu_run(name, B, cap, prec, 1)
    st, outs = oracle_run(name, B, cap, prec, 1)
    ref = outs[0]["stats"]
    got = stats[0]
    for i, nm in enumerate(STAT_NAMES):
        tol = H.stat_rtol(prec, nm, case)
        H.assert_loss(float(got[i]), float(ref[i]), nm, outs[0]["stat_scale"][i], tol)
        scale = max(abs(ref[i]), outs[0]["stat_scale"][i])
        print(f"  {nm}: gpu {got[i]:.7g} oracle {ref[i]:.7g} err/scale {abs(got[i] - ref[i]) / scale:.2e} "
              f"tol {tol:.1e}")
    assert got[7] == 0.0
    if prec == 1 and B <= 512:
        # report only: distance of the bfloat16 result from pure FP64
        _, o64 = oracle_run(name, B, cap, 0, 1)
        for i, nm in enumerate(STAT_NAMES):
            r64 = o64[0]["stats"][i]
            print(f"  bf16 vs fp64 {nm}: {abs(got[i] - r64) / max(abs(r64), 1e-30):.2e}")
    d = H.odims(name)
    blk = olayout.blocks(d)
    g = ag.grads.cpu().numpy().astype(np.float64)
    report_grads(g, outs[0], d, case)
    worst_c = H.assert_grads_per_tensor(g, outs[0]["g_enc_critic"], name, 0, 0, blk["critic"][1], case=case)
    worst_a = H.assert_grads_per_tensor(g, outs[0]["g_actor"], name, 0, blk["actor"][0], blk["actor"][1], case=case)
    la = blk["log_alpha"][0]
    la_tol = H.GRAD_RTOL if case is None else H.bf16_grad_tol(case, "log_alpha")
    assert abs(g[la] - outs[0]["g_log_alpha"][0]) <= la_tol * abs(outs[0]["g_log_alpha"][0])
    # parameters after one Adam step: a component whose gradient sign differs can
    # move by up to 2 lr, nothing more (reported, not a tolerance on the step)
    dp = np.abs(ag.params.cpu().numpy() - st.params)
    assert dp.max() <= 2 * 3e-4 * 1.001 + 1e-6
    # the target EMA takes (1 - rho) of that step: (1 - rho) 2 lr plus FP32 rounding
    dt = np.abs(ag.target.cpu().numpy() - st.target)
    assert dt.max() <= (1 - 0.995) * 2 * 3e-4 * 1.001 + 1e-6
    print(f"  worst grad (err, tol, tensor) critic {worst_c} actor {worst_a}; "
          f"param max |d| {dp.max():.2e} (mean {dp.mean():.2e}); target max |d| {dt.max():.2e}")
    counters = ag.counters.cpu().numpy()
    np.testing.assert_array_equal(counters, [1, 1, 1, 1])


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_equals_eager_and_is_deterministic(prec):
    a1, s1 = gpu_run("tiny", 32, 4096, prec, 2, graph=True, chunks=2)     # one graph replayed twice
    a2, s2 = gpu_run("tiny", 32, 4096, prec, 4, graph=False)
    a3, s3 = gpu_run("tiny", 32, 4096, prec, 2, graph=True, chunks=2)
    for x, y in ((a1, a2), (a1, a3)):
        for attr in ("params", "target", "m", "v", "counters"):
            assert torch.equal(getattr(x, attr), getattr(y, attr)), attr
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(s1, s3)


@pytest.mark.parametrize("prec", [0, 1])
def test_updates_on_the_agent_stream_equal_the_joined_path(prec):
    """Updates issued on the agent's own stream (no cross-stream joins), with the
    replay filled on another stream beforehand, give the default path's results bit for bit."""
    a1, s1 = gpu_run("tiny", 32, 4096, prec, 2, graph=True, chunks=2)
    cfg = H.cfg("tiny")
    _, rep = replay("tiny", 4096)
    a2 = api.Agent(cfg, H.params("tiny"), 32, prec=prec)
    torch.cuda.synchronize()
    s2 = [a2.sac_update(rep, 2, stream=a2.stream) for _ in range(2)]
    a2.stream.synchronize()
    s2 = torch.cat(s2).cpu().numpy()
    for attr in ("params", "target", "m", "v", "counters"):
        assert torch.equal(getattr(a1, attr), getattr(a2, attr)), attr
    np.testing.assert_array_equal(s1, s2)


def test_delayed_actor_counters_and_stats():
    ag, stats = gpu_run("tiny", 32, 4096, 0, 3, graph=True, policy_freq=2)
    np.testing.assert_array_equal(ag.counters.cpu().numpy(), [3, 3, 2, 3])
    assert stats[1, 1] == 0.0 and stats[0, 1] != 0.0 and stats[2, 1] != 0.0
    st, outs = oracle_run("tiny", 32, 4096, 0, 3, policy_freq=2)
    for u in range(3):
        assert outs[u]["actor_step"] == (u % 2 == 0)
        for i in range(7):
            H.assert_loss(float(stats[u, i]), float(outs[u]["stats"][i]), f"update {u} stat {i}",
                          outs[u]["stat_scale"][i])


def test_full_size_batch_2048_runs_and_is_finite():
    ag, stats = gpu_run("full", 2048, 4096, 1, 2, graph=True)
    assert np.all(np.isfinite(stats)) and np.all(stats[:, 7] == 0)


@pytest.mark.parametrize("name,prec", [("tiny", 0), ("full", 0), ("full", 1), ("state", 0)])
def test_act_matches_oracle(name, prec):
    cfg = H.cfg(name)
    d = H.odims(name)
    rep, grep = replay(name, 2048 if name == "full" else 4096)
    p = H.params(name)
    ag = api.Agent(cfg, p, 32, prec=prec)
    n = 300
    frames = grep["obs"][:n].contiguous()
    prop = grep["proprio"][:n].contiguous()
    hp = sac.hparams(d)
    for sample, rid in ((False, 0), (True, 12345678901)):
        a = ag.act(frames, prop, sample=sample, request_id=rid).cpu().numpy()
        ref = sac.act(p, d, hp, rep["obs"][:n], rep["proprio"][:n], sample, rid, bf=prec == 1)
        if prec == 0:
            assert np.abs(a - ref).max() < 1e-5, (sample, np.abs(a - ref).max())
        else:
            tol = H.bf16_act_tol("sample" if sample else "mean")
            e = H.rel_norm(a, ref)
            print(f"  act bf16 sample={sample}: rel-norm err {e:.2e} (tol {tol:.1e}), "
                  f"max abs {np.abs(a - ref).max():.2e}")
            assert e <= tol, (sample, e, tol)


@pytest.mark.parametrize("name,B,prec,atoms,cdq", [("tiny", 32, 0, None, True), ("tiny", 32, 0, 1, False),
                                                   ("tiny", 32, 0, 1, True), ("tiny", 32, 1, 1, False),
                                                   ("full", 512, 1, None, True), ("full", 512, 0, 1, False),
                                                   ("full", 512, 1, 1, True)])
def test_variant_update_matches_oracle(name, B, prec, atoms, cdq):
    """The paper's critic ablations (Sec. IV Critic Design Choices): the clipped
    double-Q target and the scalar critic with the squared Bellman error."""
    print(f"variant parity {name} B={B} prec={prec} atoms={atoms} cdq={cdq}", flush=True)
    cfg = dict(H.cfg(name))
    if atoms is not None:
        cfg["atoms"] = atoms
    d = olayout.dims(**cfg)
    tab = [(n, o, s) for n, (o, s) in olayout.offsets(d)[0].items()]
    p = synthetic.init_params(tab, seed=1)
    cap = 4096 if name == "tiny" else 2048
    rep, grep = replay(name, cap)
    ag = api.Agent(cfg, p, B, prec=prec, cdq=cdq)
    got = ag.sac_update(grep, 1).cpu().numpy()[0]
    hp = sac.hparams(d, cdq=cdq)
    st = sac.new_state(d, p.astype(np.float64))
    o = sac.sac_update(st, rep, d, hp, B, bf=prec == 1)
    if cdq and d.atoms > 1:
        # the twin choice is a comparison of expectations: keep it far from a tie
        z = olayout_atoms(d)
        e = np.exp(o["logits_bar"] - o["logits_bar"].max(-1, keepdims=True))
        E = (e / e.sum(-1, keepdims=True)) @ z
        assert np.min(np.abs(E[0] - E[1])) > 1e-4 * np.max(np.abs(E))
    case = None
    if prec == 1:
        case = f"{name}{'_scalar' if atoms == 1 else ''}{'_cdq' if cdq else ''}_b{B}"
    for i, nm in enumerate(STAT_NAMES):
        H.assert_loss(float(got[i]), float(o["stats"][i]), nm, o["stat_scale"][i], H.stat_rtol(prec, nm, case))
    assert got[7] == 0.0
    g = ag.grads.cpu().numpy().astype(np.float64)
    blk = olayout.blocks(d)
    report_grads(g, o, d, case)
    worst_c = H.assert_grads_per_tensor(g, o["g_enc_critic"], name, 0, 0, blk["critic"][1], case=case, dims=d)
    worst_a = H.assert_grads_per_tensor(g, o["g_actor"], name, 0, blk["actor"][0], blk["actor"][1], case=case,
                                        dims=d)
    print(f"  worst gradient (err, tol, tensor) critic {worst_c} actor {worst_a}")
    assert np.abs(ag.params.cpu().numpy() - st.params).max() <= 2 * 3e-4 * 1.001 + 1e-6
    ag.close()


def olayout_atoms(d):
    return d.v_min + np.arange(d.atoms) * ((d.v_max - d.v_min) / (d.atoms - 1))


@pytest.mark.parametrize("name,B,cap,prec", [("tiny", 32, 4096, 0), ("tiny", 32, 4096, 1), ("full", 512, 2048, 1)])
def test_optimiser_kept_encoder_weights_equal_a_fresh_preparation(name, B, cap, prec):
    """The critic Adam launch rewrites the fused encoder's rearranged weights with
    every conv weight it updates; an agent that instead re-prepares them from the
    parameters before each update (sq_agent_sync) must follow bit for bit."""
    cfg = H.cfg(name)
    _, rep = replay(name, cap)
    a = api.Agent(cfg, H.params(name), B, prec=prec)
    b = api.Agent(cfg, H.params(name), B, prec=prec)
    for _ in range(4):
        s_a = a.sac_update(rep, 1, graph=False)
        b.sync()
        s_b = b.sac_update(rep, 1, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(s_a, s_b)
    assert torch.equal(a.params, b.params) and torch.equal(a.target, b.target)


@pytest.mark.parametrize("B,prec", [(100, 0), (100, 1), (1, 0)])
def test_ragged_batch_matches_oracle(B, prec):
    """A batch that fills no tile evenly (100 rows: 3 full 32-row tiles and a
    4-row tail; 1 row: a single partial tile) through every kernel of the update."""
    name, cap = "tiny", 4096
    print(f"ragged update B={B} prec={prec}", flush=True)
    ag, stats = gpu_run(name, B, cap, prec, 1)
    st, outs = oracle_run(name, B, cap, prec, 1)
    case = f"{name}_b{B}" if prec == 1 else None
    for i, nm in enumerate(STAT_NAMES):
        H.assert_loss(float(stats[0][i]), float(outs[0]["stats"][i]), nm, outs[0]["stat_scale"][i],
                      H.stat_rtol(prec, nm, case))
    d = H.odims(name)
    blk = olayout.blocks(d)
    g = ag.grads.cpu().numpy().astype(np.float64)
    report_grads(g, outs[0], d, case)
    H.assert_grads_per_tensor(g, outs[0]["g_enc_critic"], name, 0, 0, blk["critic"][1], case=case)
    H.assert_grads_per_tensor(g, outs[0]["g_actor"], name, 0, blk["actor"][0], blk["actor"][1], case=case)


def test_degenerate_targets_match_oracle():
    """All-terminal transitions (the target collapses to the reward: a two-atom
    projection of a point) and gamma = 0 (the same target through the discount)."""
    name, B, cap = "tiny", 32, 256
    cfg = H.cfg(name)
    d = H.odims(name)
    cpu = synthetic.replay(cap, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=5, done_rate=1.0)
    assert int(cpu["done"].sum()) == cap
    rep_np = H.np_replay(cpu)
    rep = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    for gamma, rp, rg in ((0.99, rep_np, rep), (0.0, dict(rep_np, done=np.zeros_like(rep_np["done"])),
                                                dict(rep, done=torch.zeros_like(rep["done"])))):
        ag = api.Agent(cfg, H.params(name), B, gamma=gamma)
        got = ag.sac_update(rg, 1).cpu().numpy()[0]
        st = sac.new_state(d, H.params(name).astype(np.float64))
        o = sac.sac_update(st, rp, d, sac.hparams(d, gamma=gamma), B)
        # the target is the reward itself
        np.testing.assert_allclose(o["tgt"], rp["reward"][o["idx"]], rtol=1e-12, atol=1e-12)
        for i, nm in enumerate(STAT_NAMES):
            H.assert_loss(float(got[i]), float(o["stats"][i]), f"gamma {gamma} {nm}", o["stat_scale"][i])
        ag.close()


# (config, batch, replay rows, terminal rate, gamma, precision): the update's own
# mix, many and only terminal rows (every shifted atom of a row on one point), and
# gamma = 1 without terminals (the widest spread of positions)
@pytest.mark.parametrize("name,B,cap,done_rate,gamma,prec", [
    ("tiny", 32, 256, 0.01, 0.99, 0), ("tiny", 32, 256, 0.5, 0.99, 0), ("tiny", 32, 256, 1.0, 0.99, 0),
    ("tiny", 32, 256, 0.0, 1.0, 0), ("full", 512, 2048, 0.01, 0.99, 0), ("full", 512, 2048, 0.3, 0.99, 0),
    ("full", 512, 2048, 0.3, 0.99, 1)])
def test_projected_target_matches_oracle(name, B, cap, done_rate, gamma, prec):
    """The update's projected target distribution m (Eq. (1) in categorical form:
    the twin-target softmax average projected onto the support) element by
    element against the oracle's, in FP32, and invariants of the GPU's m that
    hold exactly whatever the rounding: no negative mass, each row's mass that of
    a softmax (1 up to FP32 summation), and a terminal row's mass on at most two
    adjacent atoms (all of its shifted atoms sit at the reward).  Bar for FP32:
    the positions b and the bonus -alpha log pi' carry FP32 rounding of at most
    1e-4 atoms on these supports, which moves each hat weight, and so each m_i (a
    sum of weights times probabilities that total 1), by at most that; the
    softmax adds about 1e-6."""
    print(f"projected target {name} B={B} done_rate={done_rate} gamma={gamma} prec={prec}", flush=True)
    cfg = H.cfg(name)
    d = H.odims(name)
    cpu = synthetic.replay(cap, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=11,
                           done_rate=done_rate)
    rep_np = H.np_replay(cpu)
    rep = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    ag = api.Agent(cfg, H.params(name), B, prec=prec, gamma=gamma)
    ag.sac_update(rep, 1)
    m = ag.last_target().cpu().numpy().astype(np.float64)
    idx = ag.last_indices().cpu().numpy()
    ag.close()
    assert m.shape == (B, d.atoms)
    assert np.all(np.isfinite(m)) and m.min() >= 0.0
    np.testing.assert_allclose(m.sum(axis=1), 1.0, rtol=0, atol=1e-5)
    done = rep_np["done"][idx] != 0
    for b in np.flatnonzero(done):
        nz = np.flatnonzero(m[b])
        assert 1 <= len(nz) <= 2 and nz[-1] - nz[0] <= 1, (b, nz)
    if prec == 0:
        st = sac.new_state(d, H.params(name).astype(np.float64))
        o = sac.sac_update(st, rep_np, d, sac.hparams(d, gamma=gamma), B)
        np.testing.assert_array_equal(idx, o["idx"])
        err = np.abs(m - o["m"]).max()
        print(f"  max |m - m_oracle| {err:.3e}", flush=True)
        assert err <= 1e-4 + 1e-5


@pytest.mark.parametrize("name,B,prec", [("tiny", 32, 0), ("tiny", 32, 1), ("full", 512, 1)])
def test_silent_heads_update_matches_its_closed_form(name, B, prec):
    """Zero twin critic heads, a constant actor head, all-terminal transitions and
    lr = 0: the GPU update against the closed form the oracle is pinned to (critic
    loss 2 log N, mean Q the mean atom, mean target the mean reward, head-bias
    gradient 1/N - mean two-hot(r), every other critic and encoder gradient
    exactly zero, the entropy of the constant head at the update's policy noise,
    the actor loss and the actor head-bias gradient, every other actor gradient
    exactly zero), in FP32 and BF16 (the zero head weights make the logits and the
    actor head exact in both)."""
    from tests.test_oracle_sac import head_closed_form, head_entropy, silent_heads_case, silent_heads_closed_form
    d = H.odims(name)
    cap = 256
    params, rep_np = silent_heads_case(d, cap)
    rep = {k: (torch.as_tensor(v).cuda() if isinstance(v, np.ndarray) else v) for k, v in rep_np.items()}
    hp = sac.hparams(d, lr=0.0)
    rows = philox.sample_indices(hp.seed, 0, cap, B)
    blk = olayout.blocks(d)
    cf = silent_heads_closed_form(d, rep_np, rows, float(np.exp(params[blk["log_alpha"][0]])))
    ag = api.Agent(H.cfg(name), params.astype(np.float32), B, prec=prec, lr=0.0)
    s = ag.sac_update(rep, 1).cpu().numpy()[0].astype(np.float64)
    np.testing.assert_array_equal(ag.last_indices().cpu().numpy(), rows)
    g = ag.grads.cpu().numpy().astype(np.float64)
    ag.close()
    print(f"  {name} B={B} prec={prec}: loss {s[0]:.9g} (2 log N {cf['loss']:.9g}), mean Q {s[5]:.3g}, "
          f"mean target {s[6]:.9g} ({cf['mean_target']:.9g})")
    assert abs(s[0] - cf["loss"]) <= 1e-6 * cf["loss"]
    assert abs(s[5] - cf["mean_q"]) <= 1e-6 * (abs(d.v_min) + abs(d.v_max))
    assert abs(s[6] - cf["mean_target"]) <= 1e-6
    ent = head_entropy(d, hp, B)
    assert abs(s[4] - ent) <= 1e-5 * abs(ent)
    assert abs(s[2] - cf["alpha0"] * (ent - hp.target_entropy)) <= 1e-5 * abs(s[2]) + 1e-7
    # lr = 0: the actor loss and the actor gradient against the still-silent critic
    assert abs(s[1] - (-cf["alpha0"] * ent - cf["mean_q"])) <= 1e-5 * abs(cf["alpha0"] * ent)
    for n, (off, shp) in olayout.offsets(d)[0].items():
        if not n.startswith("actor."):
            continue
        k = int(np.prod(shp))
        if n == "actor.out.b":
            ref = head_closed_form(d, hp, B, cf["alpha0"])
            assert H.rel_norm(g[off:off + k], ref) <= 1e-5, n
        elif n != "actor.out.W":
            assert np.all(g[off:off + k] == 0.0), n
    for n, (off, shp) in olayout.offsets(d)[0].items():
        if off >= blk["critic"][1]:
            continue
        k = int(np.prod(shp))
        if n in ("q1.out.b", "q2.out.b"):
            np.testing.assert_allclose(g[off:off + k], cf["g_bias"], rtol=0, atol=1e-6, err_msg=n)
        elif n not in ("q1.out.W", "q2.out.W"):
            assert np.all(g[off:off + k] == 0.0), n


@pytest.mark.parametrize("name,B,prec", [("tiny", 32, 0), ("full", 512, 1)])
def test_silent_heads_soft_target_matches_its_closed_form(name, B, prec):
    """Non-terminal transitions, silent critic heads, gamma = 1/4: the mean target
    is mean_b (r_b + gamma (mean z - alpha log pi'_b)) with log pi' the constant
    actor head's density at the noise of the sample at s_t+1 (the closed form the
    oracle is pinned to), and the critic loss 2 log N."""
    from tests.test_oracle_sac import head_logp, silent_heads_case
    d = H.odims(name)
    cap = 256
    params, rep_np = silent_heads_case(d, cap, terminal=False)
    rep = {k: (torch.as_tensor(v).cuda() if isinstance(v, np.ndarray) else v) for k, v in rep_np.items()}
    hp = sac.hparams(d, gamma=0.25)
    rows = philox.sample_indices(hp.seed, 0, cap, B)
    alpha0 = float(np.exp(params[olayout.blocks(d)["log_alpha"][0]]))
    r = rep_np["reward"][rows].astype(np.float64)
    z = np.linspace(d.v_min, d.v_max, d.atoms)
    want = float(np.mean(r + hp.gamma * (z.mean() - alpha0 * head_logp(d, hp, B, 1))))
    ag = api.Agent(H.cfg(name), params.astype(np.float32), B, prec=prec, gamma=0.25)
    s = ag.sac_update(rep, 1).cpu().numpy()[0].astype(np.float64)
    ag.close()
    print(f"  {name} B={B} prec={prec}: mean target {s[6]:.9g} (closed form {want:.9g}), loss {s[0]:.9g}")
    assert abs(s[6] - want) <= 1e-5 * (abs(want) + 1.0)
    assert abs(s[0] - 2.0 * math.log(d.atoms)) <= 1e-6 * s[0]


@pytest.mark.parametrize("name,B,cap", [("tiny", 32, 4096), ("full", 512, 2048), ("state", 512, 2048)])
def test_utd_block_matches_oracle(name, B, cap):
    """Alg. 1's inner loop inside captured graphs, against the oracle's updates
    u = 0..3 from the same initial state: every update's replay rows (drawn on the
    device from the update counter) equal the oracle's Philox draw bit for bit,
    and every update's statistics match.  One agent replays a one-update graph
    four times (rows checked after each), another runs one four-update graph."""
    print(f"UTD block {name} B={B}", flush=True)
    cfg = H.cfg(name)
    rep_np, rep = replay(name, cap)
    st, outs = oracle_run(name, B, cap, 0, 4)
    a1 = api.Agent(cfg, H.params(name), B)
    s1 = []
    for u in range(4):
        s1.append(a1.sac_update(rep, 1, stream=a1.stream))
        idx = a1.last_indices().cpu().numpy()
        np.testing.assert_array_equal(idx, philox.sample_indices(2, u, cap, B), err_msg=f"update {u}")
        np.testing.assert_array_equal(idx, outs[u]["idx"])
    assert a1.graph_count() == (1, 1)
    a4 = api.Agent(cfg, H.params(name), B)
    s4 = a4.sac_update(rep, 4, stream=a4.stream)
    np.testing.assert_array_equal(a4.last_indices().cpu().numpy(), outs[3]["idx"])
    s1 = torch.cat(s1).cpu().numpy()
    s4 = s4.cpu().numpy()
    # the two paths run the same kernels in the same order
    np.testing.assert_array_equal(s1, s4)
    for u in range(4):
        for i, nm in enumerate(STAT_NAMES):
            ref = outs[u]["stats"][i]
            scale = max(abs(ref), outs[u]["stat_scale"][i])
            print(f"  u={u} {nm}: gpu {s4[u, i]:.7g} oracle {ref:.7g} err/scale {abs(s4[u, i] - ref) / scale:.2e}")
            H.assert_loss(float(s4[u, i]), float(ref), f"update {u} {nm}", outs[u]["stat_scale"][i])
        assert s4[u, 7] == 0.0
    np.testing.assert_array_equal(a4.counters.cpu().numpy(), [4, 4, 4, 4])
    # each update moves a parameter by at most lr from Adam's normalised step, so
    # after four updates a component whose gradient sign flipped differs by < 8 lr
    dp = np.abs(a4.params.cpu().numpy() - st.params)
    print(f"  params after 4 updates: max |d| {dp.max():.2e}, mean {dp.mean():.2e}")
    assert dp.max() <= 8 * 3e-4 * 1.001
    a1.close()
    a4.close()


def test_non_finite_update_sets_the_health_flag():
    """A NaN reward at a row drawn by update 0 makes that row's projected target
    NaN (as the clamp of the projection's definition keeps it), so the critic
    loss and the mean target are NaN and stats[0, 7] = 1, on both sides."""
    name, B, cap = "tiny", 32, 4096
    cfg = H.cfg(name)
    d = H.odims(name)
    cpu = synthetic.replay(cap, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0)
    rows = philox.sample_indices(2, 0, cap, B)
    cpu["reward"][torch.as_tensor(rows[:3].astype(np.int64))] = float("nan")
    rep_np = H.np_replay(cpu)
    rep = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    for prec in (0, 1):
        ag = api.Agent(cfg, H.params(name), B, prec=prec)
        got = ag.sac_update(rep, 1).cpu().numpy()[0]
        st = sac.new_state(d, H.params(name).astype(np.float64))
        o = sac.sac_update(st, rep_np, d, sac.hparams(d), B, bf=prec == 1)
        print(f"  prec {prec}: gpu {got}, oracle {o['stats']}")
        assert o["stats"][7] == 1.0 and got[7] == 1.0
        np.testing.assert_array_equal(np.isnan(got[:7]), np.isnan(o["stats"][:7]))
        # the critic and encoder took the non-finite step (the caller restores them)
        c0, c1 = olayout.blocks(d)["critic"]
        assert not np.isfinite(ag.params[c0:c1].cpu().numpy()).all()
        ag.close()


def test_graph_cache_keys_on_replay_contents_not_padding_or_stats():
    """Two replay structs that differ only in their padding bytes, and a fresh
    stats buffer on every call, replay one captured graph; a replay whose size
    grew is a new key, and its rows are drawn over the new size."""
    import ctypes

    from paper_2602_21203_amd import _lib

    name, B, cap = "tiny", 32, 4096
    cfg = H.cfg(name)
    _, rep = replay(name, cap)
    ag = api.Agent(cfg, H.params(name), B)
    rs = api.replay_struct(rep)
    raw = bytearray(bytes(rs))
    pad = _lib.Replay.dev_size.offset - (_lib.Replay.squinted.offset + ctypes.sizeof(ctypes.c_int))
    assert pad > 0
    for i in range(_lib.Replay.squinted.offset + 4, _lib.Replay.dev_size.offset):
        raw[i] = 0xAB
    rs2 = _lib.Replay.from_buffer_copy(raw)
    assert bytes(rs2) != bytes(rs)
    st = ag.stream
    for r in (rs, rs2, rs, rs2):
        stats = torch.empty((2, 8), dtype=torch.float32, device="cuda")
        _lib.check(_lib.LIB.sac_update(ag.handle, ctypes.byref(r), 2, _lib.ptr(stats), _lib.stream_handle(st)))
        st.synchronize()
        assert np.isfinite(stats.cpu().numpy()).all()
    assert ag.graph_count() == (1, 1)
    # the Python path builds a fresh struct and stats tensor per call: same graph
    for _ in range(3):
        ag.sac_update(rep, 2, stream=st)
    assert ag.graph_count() == (1, 1)
    # a smaller row count is another key; the draw follows it (updates 14 and 15)
    small = dict(rep, size=100)
    ag.sac_update(small, 2, stream=st)
    assert ag.graph_count() == (2, 2)
    np.testing.assert_array_equal(ag.last_indices().cpu().numpy(), philox.sample_indices(2, 15, 100, B))
    # beyond 8 graphs the least recently used one is evicted
    for n in range(3, 12):
        ag.sac_update(rep, n, stream=st)
    captured, cached = ag.graph_count()
    assert captured == 11 and cached == 8
    st.synchronize()
    assert int(ag.counters[0]) == 4 * 2 + 3 * 2 + 2 + sum(range(3, 12))
    ag.close()
