"""One Squint SAC update in FP64, following Alg. 1 in the paper's order.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

An update u (Alg. 1, inner loop; Sec. III Eqs. (1)-(3); Sec. IV design
choices) performs, in order:
  1. draw B replay indices and the two Gaussian noise blocks (philox)
  2. squint obs and next_obs of the sampled rows (squint)
  3. encode both halves with the current encoder (same psi for z_t, z_{t+1})
  4. target: a' ~ pi(z_{t+1}, s'), average the softmaxed twin target critics,
     shift every atom by -alpha log pi(a'), discount, project onto the atoms
     (variants: the clipped double-Q target takes, per row, the twin with the
     smaller expected value; a scalar critic, atoms = 1, uses Eq. (1) directly)
  5. critic + encoder: cross entropy of both online critics to the target
     (scalar critic: Eq. (2), the squared error), backward into the critic and
     the encoder, one Adam step on (psi, theta)
  6. temperature: a ~ pi(stopgrad z_t, s) with fresh noise; gradient of
     alpha * mean(-log pi - H_target) with respect to log alpha; Adam on log alpha
  7. actor (when u % policy_freq == 0): the updated critic scores a; loss
     mean(alpha_new log pi - (Q1 + Q2) / 2); backward through the critic into
     the action only, then through the policy; Adam on phi
  8. target critic EMA with the updated theta
Readings (also in the design notes): the temperature loss sign is the one of
Haarnoja et al. (the paper's Alg. 1 line is garbled); Adam with bias
correction for all three optimisers, each with its own step count; the actor
uses the pre-update conv features and the post-update critic; the delayed actor
test uses the global update counter u.

Stats row (8 values): critic loss, actor loss (0 when the actor is not
stepped), temperature loss, alpha after the update, mean entropy estimate
-log pi, mean expected Q of the online critics at the replayed actions
(averaged over twins), mean expected value of the projected target, and a
non-finite flag (1 if any of the first seven is NaN or Inf).
"""
from types import SimpleNamespace

import numpy as np

from . import layout, nets, philox
from .squint import squint

HP_DEFAULT = dict(gamma=0.99, lr=3e-4, beta1=0.9, beta2=0.999, adam_eps=1e-8, rho=0.995,
                  target_entropy=None, log_std_min=-5.0, log_std_max=2.0, policy_freq=1, seed=2, cdq=False)


def hparams(d, **kw):
    hp = dict(HP_DEFAULT)
    hp.update(kw)
    if hp["target_entropy"] is None:
        hp["target_entropy"] = -float(d.action)
    return SimpleNamespace(**hp)


def adam(p, g, m, v, t, hp):
    """Adam with bias correction; t is the step count after increment."""
    m[:] = hp.beta1 * m + (1.0 - hp.beta1) * g
    v[:] = hp.beta2 * v + (1.0 - hp.beta2) * g * g
    mhat = m / (1.0 - hp.beta1 ** t)
    vhat = v / (1.0 - hp.beta2 ** t)
    p[:] = p - hp.lr * mhat / (np.sqrt(vhat) + hp.adam_eps)


def ema(target, online, rho):
    target[:] = rho * target + (1.0 - rho) * online


def new_state(d, params):
    """Fresh optimiser state: target = critic block, zero moments, zero counters."""
    params = np.asarray(params, dtype=np.float64).copy()
    c0, c1 = layout.blocks(d)["critic"]
    return SimpleNamespace(params=params, target=params[c0:c1].copy(),
                           m=np.zeros_like(params), v=np.zeros_like(params),
                           steps=np.zeros(3, dtype=np.int64), u=0)


def copy_state(s):
    return SimpleNamespace(params=s.params.copy(), target=s.target.copy(), m=s.m.copy(),
                           v=s.v.copy(), steps=s.steps.copy(), u=s.u)


def _flatten(grads, d, block):
    table, total = layout.offsets(d)
    out = np.zeros(total)
    for name, g in grads.items():
        o, shp = table[name]
        out[o:o + g.size] = g.ravel()
    a, b = layout.blocks(d)[block] if isinstance(block, str) else block
    return out[a:b]


def gather_batch(replay, idx):
    return {k: np.asarray(replay[k])[idx] for k in
            ("obs", "next_obs", "proprio", "next_proprio", "action", "reward", "done")}


def sac_update(state, replay, d, hp, batch, bf=False):
    """Advance `state` (modified in place) by one update; returns diagnostics."""
    u = state.u
    B, A = batch, d.action
    blk = layout.blocks(d)
    P = layout.view(state.params, d)

    # 1. minibatch and noise
    idx = philox.sample_indices(hp.seed, u, replay["size"], B)
    eps_next = philox.gaussian(hp.seed, u, 1, B * A).reshape(B, A)
    eps = philox.gaussian(hp.seed, u, 2, B * A).reshape(B, A)
    bt = gather_batch(replay, idx)
    s, s2 = bt["proprio"].astype(np.float64), bt["next_proprio"].astype(np.float64)
    a_rep = bt["action"].astype(np.float64)
    r = bt["reward"].astype(np.float64)
    done = bt["done"].astype(np.float64)

    # 2-3. squint and encode both halves with the current encoder
    # (frames stored already squinted, as by squint at insertion, carry k = 1);
    # state-based SAC (no encoder) uses the states themselves as the features
    image = d.n_conv > 0
    if image:
        k = replay.get("k", d.k)
        x = np.concatenate([squint(bt["obs"], k), squint(bt["next_obs"], k)])
        feat, enc_cache = nets.encoder_fwd(P, x, d.n_conv, bf)
    else:
        x = None
        feat = np.concatenate([s, s2])
    f_t, f_n = feat[:B], feat[B:]

    # 4. soft target: distributional (C51, atoms >= 2) or scalar (atoms == 1, Eq. (1));
    # the twin targets are averaged, or the smaller one is taken (clipped double-Q)
    alpha = float(np.exp(P["log_alpha"][0]))
    a_n, logp_n, _ = nets.actor_fwd(P, f_n, s2, eps_next, hp.log_std_min, hp.log_std_max, bf)
    T = layout.target_view(state.target, d)
    logits_bar, _ = nets.critic_fwd(T, f_n, s2, a_n, bf)
    bonus = -alpha * logp_n
    scalar = d.atoms == 1
    if scalar:
        qbar = logits_bar[:, :, 0]
        q_next = np.minimum(qbar[0], qbar[1]) if hp.cdq else 0.5 * (qbar[0] + qbar[1])
        y = r + hp.gamma * (1.0 - done) * (q_next + bonus)
        m, z, tgt = y[:, None], np.ones(1), y
    else:
        if hp.cdq:
            p_bar, _ = nets.cdq_select(logits_bar, nets.atoms(d.atoms, d.v_min, d.v_max))
        else:
            p_bar = 0.5 * (nets.softmax(logits_bar[0]) + nets.softmax(logits_bar[1]))
        m = nets.c51_project(p_bar, r, done, hp.gamma, bonus, d.v_min, d.v_max)
        z = nets.atoms(d.atoms, d.v_min, d.v_max)
        tgt = m @ z

    # 5. critic + encoder step: cross entropy to m (C51) or Eq. (2) to y (scalar)
    logits, ccache = nets.critic_fwd(P, f_t, s, a_rep, bf)
    if scalar:
        q_rep = logits[:, :, 0]
        loss_c, dq_c = nets.mse_loss(q_rep, y)
        dlogits = dq_c[:, :, None]
    else:
        loss_c, dlogits = nets.cross_entropy(logits, m)
        q_rep, _ = nets.expected_q(logits, z)
    g_critic, dfeat_t, _ = nets.critic_bwd(P, ccache, dlogits, bf)
    g_all = dict(g_critic)
    if image:
        dfeat = np.concatenate([dfeat_t, np.zeros_like(f_n)])
        g_all.update(nets.encoder_bwd(P, enc_cache, dfeat, d.n_conv, bf))
    g_ec = _flatten(g_all, d, (blk["enc"][0], blk["critic"][1]))
    lo, hi = blk["enc"][0], blk["critic"][1]
    state.steps[0] += 1
    adam(state.params[lo:hi], g_ec, state.m[lo:hi], state.v[lo:hi], state.steps[0], hp)

    # 6. temperature step (actor sample on stop-gradient pre-update features)
    a_t, logp_t, acache = nets.actor_fwd(P, f_t, s, eps, hp.log_std_min, hp.log_std_max, bf)
    ent_gap = float(np.mean(-logp_t - hp.target_entropy))
    loss_alpha = alpha * ent_gap
    g_la = np.array([alpha * ent_gap])
    la = slice(*blk["log_alpha"])
    state.steps[2] += 1
    adam(state.params[la], g_la, state.m[la], state.v[la], state.steps[2], hp)
    alpha_new = float(np.exp(state.params[la][0]))

    # 7. delayed actor step against the updated critic
    loss_pi = 0.0
    g_actor = np.zeros(blk["actor"][1] - blk["actor"][0])
    actor_step = (u % hp.policy_freq) == 0
    if actor_step:
        Pn = layout.view(state.params, d)
        logits_q, qcache = nets.critic_fwd(Pn, f_t, s, a_t, bf)
        if scalar:
            q, dq = logits_q[:, :, 0], np.ones_like(logits_q)
        else:
            q, dq = nets.expected_q(logits_q, z)
        loss_pi = float(np.mean(alpha_new * logp_t - 0.5 * (q[0] + q[1])))
        dlogits_q = -0.5 / B * dq
        _, _, da = nets.critic_bwd(Pn, qcache, dlogits_q, bf, need_params=False, need_dfeat=False)
        g_act = nets.actor_bwd(P, acache, da, np.full(B, alpha_new / B), bf)
        g_actor = _flatten(g_act, d, "actor")
        ac = slice(*blk["actor"])
        state.steps[1] += 1
        adam(state.params[ac], g_actor, state.m[ac], state.v[ac], state.steps[1], hp)

    # 8. target EMA over the critic block
    ema(state.target, state.params[slice(*blk["critic"])], hp.rho)

    stats = np.array([loss_c, loss_pi, loss_alpha, alpha_new, float(np.mean(-logp_t)),
                      float(np.mean(q_rep)), float(np.mean(tgt)), 0.0])
    stats[7] = 0.0 if np.all(np.isfinite(stats[:7])) else 1.0
    # magnitude of the terms each statistic averages: a mean of signed terms can
    # sit near zero, so its rounding error scales with these, not with the mean
    qa = 0.5 * (q[0] + q[1]) if actor_step else np.zeros(B)
    stat_scale = np.array([abs(loss_c), float(np.mean(np.abs(alpha_new * logp_t) + np.abs(qa))),
                           alpha * float(np.mean(np.abs(-logp_t - hp.target_entropy))), abs(alpha_new),
                           float(np.mean(np.abs(logp_t))), float(np.mean(np.abs(q_rep))),
                           float(np.mean(np.abs(tgt)))])
    state.u = u + 1
    return dict(idx=idx, eps_next=eps_next, eps=eps, x=x, feat=feat, m=m, tgt=tgt, logits_bar=logits_bar,
                logits=logits,
                dlogits=dlogits, g_enc_critic=g_ec, g_log_alpha=g_la, g_actor=g_actor,
                stats=stats, stat_scale=stat_scale, actor_step=actor_step, a_next=a_n, logp_next=logp_n,
                a_t=a_t, logp_t=logp_t)


def act(params, d, hp, frames, proprio, sample, request_id=0, bf=False):
    """Policy query of Alg. 1 (sample a_t from pi(f(squint(o)), s)): mean or sampled action."""
    P = layout.view(np.asarray(params, dtype=np.float64), d)
    s = np.asarray(proprio, dtype=np.float64)
    if d.n_conv > 0:
        f, _ = nets.encoder_fwd(P, squint(frames, d.k), d.n_conv, bf)
    else:
        f = s
    if not sample:
        a, _, _ = nets.actor_fwd(P, f, s, None, hp.log_std_min, hp.log_std_max, bf)
        return a
    eps = philox.act_noise(hp.seed, request_id, f.shape[0], d.action)
    a, _, _ = nets.actor_fwd(P, f, s, eps, hp.log_std_min, hp.log_std_max, bf)
    return a
