"""Network pieces of the Squint agent in FP64, forward and hand-written backward.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sources in the paper:
  encoder      Sec. III (shared CNN encoder f_psi trained by the critic) and
               Sec. IV Encoder Design Choices (small conv encoder shared by actor
               and critic, separate one-layer projections per head)
  LayerNorm    Sec. IV Normalization (every linear layer is followed by LN)
  C51 critic   Sec. IV Critic Design Choices (categorical critic trained by
               cross entropy; the twin targets are averaged, not min-ed)
  actor        Sec. III Eq. (3) (stochastic policy, reparameterised sample)
  target       Eq. (1) and Alg. 1 (soft Bellman target from the averaged twin
               target critics); the categorical form follows Bellemare et al.

Readings where the paper is silent (each also listed in the design notes):
  convs are 3x3 valid, first stride 2, ReLU after each; LN eps 1e-5 with
  biased variance and learnable affine; no LN on output heads; the critic input
  is [h_c; proprio; action], the actor input [h_a; proprio]; the policy
  log-std is squashed smoothly, log sigma = lo + (hi - lo)(tanh(u_s) + 1)/2;
  the categorical projection uses the hat-function form with the atom position
  clamped to [0, N-1]; the entropy bonus shifts every atom.

`bf` selects the bfloat16-operand mode: every GEMM / convolution operand
(weights, activations, and upstream gradients in backward) is rounded to the
nearest bfloat16 before an FP64 product.  Bias, LayerNorm-parameter gradients
and every non-GEMM step use the unrounded values.
"""
import numpy as np

from .bf16 import maybe, maybe_computed

LN_EPS = 1e-5
LOG_2PI = float(np.log(2.0 * np.pi))
LOG_2 = float(np.log(2.0))


# ---------------------------------------------------------------- convolution
def _out(n, stride):
    return (n - 3) // stride + 1


def conv_fwd(x, W, b, stride, bf=False):
    """Valid 3x3 convolution, NCHW input, W [F, C, 3, 3]."""
    xb, Wb = maybe_computed(x, bf), maybe(W, bf)
    n, _, H, Wd = x.shape
    Ho, Wo = _out(H, stride), _out(Wd, stride)
    y = np.zeros((n, W.shape[0], Ho, Wo))
    for i in range(3):
        for j in range(3):
            patch = xb[:, :, i:i + stride * (Ho - 1) + 1:stride, j:j + stride * (Wo - 1) + 1:stride]
            y += np.einsum("ncyx,fc->nfyx", patch, Wb[:, :, i, j], optimize=True)
    return y + b[None, :, None, None]


def conv_bwd(dy, x, W, stride, bf=False, need_dx=True):
    """Gradients of conv_fwd: (dx or None, dW, db)."""
    dyb, xb, Wb = maybe_computed(dy, bf), maybe_computed(x, bf), maybe(W, bf)
    Ho, Wo = dy.shape[2], dy.shape[3]
    dW = np.zeros(W.shape)
    dx = np.zeros(x.shape) if need_dx else None
    for i in range(3):
        for j in range(3):
            sl = (slice(None), slice(None),
                  slice(i, i + stride * (Ho - 1) + 1, stride), slice(j, j + stride * (Wo - 1) + 1, stride))
            dW[:, :, i, j] = np.einsum("nfyx,ncyx->fc", dyb, xb[sl], optimize=True)
            if need_dx:
                dx[sl] += np.einsum("nfyx,fc->ncyx", dyb, Wb[:, :, i, j], optimize=True)
    return dx, dW, dy.sum(axis=(0, 2, 3))


# ---------------------------------------------------------------- dense layers
def linear(x, W, b, bf=False):
    return maybe_computed(x, bf) @ maybe(W, bf).T + b


def linear_bwd(dy, x, W, bf=False, need_dx=True):
    dyb = maybe_computed(dy, bf)
    dW = dyb.T @ maybe_computed(x, bf)
    dx = dyb @ maybe(W, bf) if need_dx else None
    return dx, dW, dy.sum(axis=0)


def ln_fwd(x, g, b):
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + LN_EPS)
    xh = (x - mu) * rstd
    return g * xh + b, (xh, rstd)


def ln_bwd(dy, cache, g):
    xh, rstd = cache
    dxh = dy * g
    dx = rstd * (dxh - dxh.mean(axis=-1, keepdims=True)
                 - xh * (dxh * xh).mean(axis=-1, keepdims=True))
    return dx, (dy * xh).sum(axis=0), dy.sum(axis=0)


def dense_ln_act(x, W, b, g, beta, act, bf=False):
    """Linear -> LayerNorm -> tanh | relu."""
    z, lnc = ln_fwd(linear(x, W, b, bf), g, beta)
    y = np.tanh(z) if act == "tanh" else np.maximum(z, 0.0)
    return y, (x, W, g, lnc, y, act)


def dense_ln_act_bwd(dy, cache, bf=False, need_dx=True):
    """Returns (dx, dW, db, dg, dbeta)."""
    x, W, g, lnc, y, act = cache
    dz = dy * (1.0 - y * y) if act == "tanh" else dy * (y > 0.0)
    dpre, dg, dbeta = ln_bwd(dz, lnc, g)
    dx, dW, db = linear_bwd(dpre, x, W, bf, need_dx)
    return dx, dW, db, dg, dbeta


# ---------------------------------------------------------------- encoder
def encoder_fwd(P, x, n_conv, bf=False):
    """Shared conv encoder; returns features flattened in (channel, y, x) order."""
    h, caches = x, []
    for i in range(n_conv):
        stride = 2 if i == 0 else 1
        out = np.maximum(conv_fwd(h, P[f"enc.conv{i + 1}.W"], P[f"enc.conv{i + 1}.b"], stride, bf), 0.0)
        caches.append((h, out, stride))
        h = out
    return h.reshape(h.shape[0], -1), caches


def encoder_bwd(P, caches, dfeat, n_conv, bf=False):
    """Encoder parameter gradients {name: grad}; no gradient to the image."""
    grads = {}
    dh = dfeat.reshape(caches[-1][1].shape)
    for i in reversed(range(n_conv)):
        h_in, out, stride = caches[i]
        dpre = dh * (out > 0.0)
        dh, dW, db = conv_bwd(dpre, h_in, P[f"enc.conv{i + 1}.W"], stride, bf, need_dx=i > 0)
        grads[f"enc.conv{i + 1}.W"] = dW
        grads[f"enc.conv{i + 1}.b"] = db
    return grads


# ---------------------------------------------------------------- critic
def critic_fwd(P, f, s, a, bf=False):
    """Twin C51 critics sharing the critic projection: logits [2, n, atoms]."""
    h, ct = dense_ln_act(f, P["critic.trunk.W"], P["critic.trunk.b"],
                         P["critic.trunk.ln.g"], P["critic.trunk.ln.b"], "tanh", bf)
    X1 = np.concatenate([h, s, a], axis=1)
    logits, qc = [], []
    for q in ("q1", "q2"):
        g1, c1 = dense_ln_act(X1, P[q + ".l1.W"], P[q + ".l1.b"], P[q + ".l1.ln.g"], P[q + ".l1.ln.b"], "relu", bf)
        g2, c2 = dense_ln_act(g1, P[q + ".l2.W"], P[q + ".l2.b"], P[q + ".l2.ln.g"], P[q + ".l2.ln.b"], "relu", bf)
        logits.append(linear(g2, P[q + ".out.W"], P[q + ".out.b"], bf))
        qc.append((c1, c2, g2))
    return np.stack(logits), (ct, qc, h.shape[1], s.shape[1])


def critic_bwd(P, cache, dlogits, bf=False, need_params=True, need_dfeat=True):
    """Backward of critic_fwd.  Returns (grads dict or None, dfeat or None, daction)."""
    ct, qc, proj, P_dim = cache
    grads = {} if need_params else None
    dX1 = 0.0
    for i, q in enumerate(("q1", "q2")):
        c1, c2, g2 = qc[i]
        dg2, dWo, dbo = linear_bwd(dlogits[i], g2, P[q + ".out.W"], bf)
        dg1, dW2, db2, dg2g, dg2b = dense_ln_act_bwd(dg2, c2, bf)
        dx1, dW1, db1, dg1g, dg1b = dense_ln_act_bwd(dg1, c1, bf)
        dX1 = dX1 + dx1
        if need_params:
            grads.update({q + ".out.W": dWo, q + ".out.b": dbo,
                          q + ".l2.W": dW2, q + ".l2.b": db2, q + ".l2.ln.g": dg2g, q + ".l2.ln.b": dg2b,
                          q + ".l1.W": dW1, q + ".l1.b": db1, q + ".l1.ln.g": dg1g, q + ".l1.ln.b": dg1b})
    daction = dX1[:, proj + P_dim:]
    dfeat = None
    if need_params or need_dfeat:
        df, dWt, dbt, dgt, dbtb = dense_ln_act_bwd(dX1[:, :proj], ct, bf, need_dx=need_dfeat)
        dfeat = df
        if need_params:
            grads.update({"critic.trunk.W": dWt, "critic.trunk.b": dbt,
                          "critic.trunk.ln.g": dgt, "critic.trunk.ln.b": dbtb})
    return grads, dfeat, daction


# ---------------------------------------------------------------- actor
def softplus(x):
    return np.logaddexp(0.0, x)


def actor_fwd(P, f, s, eps, log_std_min, log_std_max, bf=False):
    """Tanh-Gaussian policy.  eps None -> deterministic action tanh(mu).

    Returns (action, log_pi or None, cache)."""
    h, ct = dense_ln_act(f, P["actor.trunk.W"], P["actor.trunk.b"],
                         P["actor.trunk.ln.g"], P["actor.trunk.ln.b"], "tanh", bf)
    X1 = np.concatenate([h, s], axis=1)
    g1, c1 = dense_ln_act(X1, P["actor.l1.W"], P["actor.l1.b"], P["actor.l1.ln.g"], P["actor.l1.ln.b"], "relu", bf)
    g2, c2 = dense_ln_act(g1, P["actor.l2.W"], P["actor.l2.b"], P["actor.l2.ln.g"], P["actor.l2.ln.b"], "relu", bf)
    out = linear(g2, P["actor.out.W"], P["actor.out.b"], bf)
    A = out.shape[1] // 2
    mu, us = out[:, :A], out[:, A:]
    if eps is None:
        return np.tanh(mu), None, None
    tus = np.tanh(us)
    log_std = log_std_min + 0.5 * (log_std_max - log_std_min) * (tus + 1.0)
    std = np.exp(log_std)
    u = mu + std * eps
    a = np.tanh(u)
    # Gaussian log-density of u (its standardised value is eps) plus the log
    # Jacobian of the tanh squash, log(1 - tanh(u)^2) = 2 (log 2 - u - softplus(-2u)).
    logp = np.sum(-0.5 * eps * eps - log_std - 0.5 * LOG_2PI
                  - 2.0 * (LOG_2 - u - softplus(-2.0 * u)), axis=1)
    cache = (ct, c1, c2, g2, tus, std, eps, a, h.shape[1], log_std_max - log_std_min)
    return a, logp, cache


def actor_bwd(P, cache, da, dlogp, bf=False):
    """Actor parameter gradients from d action [n, A] and d log_pi [n]."""
    ct, c1, c2, g2, tus, std, eps, a, proj, span = cache
    dlogp = dlogp[:, None]
    du = da * (1.0 - a * a) + dlogp * 2.0 * a   # d log_pi / du = 2 tanh(u)
    dlog_std = du * std * eps - dlogp
    dus = dlog_std * 0.5 * span * (1.0 - tus * tus)
    dout = np.concatenate([du, dus], axis=1)
    grads = {}
    dg2, grads["actor.out.W"], grads["actor.out.b"] = linear_bwd(dout, g2, P["actor.out.W"], bf)
    dg1, grads["actor.l2.W"], grads["actor.l2.b"], grads["actor.l2.ln.g"], grads["actor.l2.ln.b"] = \
        dense_ln_act_bwd(dg2, c2, bf)
    dX1, grads["actor.l1.W"], grads["actor.l1.b"], grads["actor.l1.ln.g"], grads["actor.l1.ln.b"] = \
        dense_ln_act_bwd(dg1, c1, bf)
    _, grads["actor.trunk.W"], grads["actor.trunk.b"], grads["actor.trunk.ln.g"], grads["actor.trunk.ln.b"] = \
        dense_ln_act_bwd(dX1[:, :proj], ct, bf, need_dx=False)
    return grads


# ---------------------------------------------------------------- C51 heads
def softmax(x):
    e = np.exp(x - x.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def log_softmax(x):
    s = x - x.max(axis=-1, keepdims=True)
    return s - np.log(np.exp(s).sum(axis=-1, keepdims=True))


def atoms(n, v_min, v_max):
    return v_min + np.arange(n) * ((v_max - v_min) / (n - 1))


def c51_project(p, reward, done, gamma, bonus, v_min, v_max):
    """Categorical projection of the shifted, discounted support onto the atoms.

    Tz_j = r + gamma (1 - d)(z_j + bonus); b_j = clamp((Tz_j - v_min)/dz, 0, N-1);
    m_i = sum_j p_j max(0, 1 - |b_j - i|)."""
    n_at = p.shape[1]
    dz = (v_max - v_min) / (n_at - 1)
    z = atoms(n_at, v_min, v_max)
    Tz = reward[:, None] + gamma * (1.0 - done[:, None]) * (z[None, :] + bonus[:, None])
    b = np.clip((Tz - v_min) / dz, 0.0, n_at - 1)
    hat = np.maximum(0.0, 1.0 - np.abs(b[:, :, None] - np.arange(n_at)[None, None, :]))
    return np.einsum("bj,bji->bi", p, hat)


def c51_project_scatter(p, reward, done, gamma, bonus, v_min, v_max):
    """The textbook floor/ceil scatter form (lower == upper handled by giving the
    whole mass to that atom).  Used only to pin c51_project."""
    n, n_at = p.shape
    dz = (v_max - v_min) / (n_at - 1)
    z = atoms(n_at, v_min, v_max)
    m = np.zeros_like(p)
    for r in range(n):
        for j in range(n_at):
            tz = reward[r] + gamma * (1.0 - done[r]) * (z[j] + bonus[r])
            tz = min(max(tz, v_min), v_max)
            bj = (tz - v_min) / dz
            lo, hi = int(np.floor(bj)), int(np.ceil(bj))
            if lo == hi:
                m[r, lo] += p[r, j]
            else:
                m[r, lo] += p[r, j] * (hi - bj)
                m[r, hi] += p[r, j] * (bj - lo)
    return m


def cross_entropy(logits, m):
    """Sum over the twins of the batch-mean CE to the projected target m.

    Returns (loss, dlogits) with dlogits = (softmax - m) / n."""
    n = m.shape[0]
    loss = float(np.sum(-np.sum(m[None] * log_softmax(logits), axis=-1).mean(axis=1)))
    return loss, (softmax(logits) - m[None]) / n


def expected_q(logits, z):
    """Q_i = sum_j softmax(l_i)_j z_j and its gradient dQ_i / dl_ij = p_ij (z_j - Q_i)."""
    p = softmax(logits)
    q = p @ z
    return q, p * (z - q[..., None])


def cdq_select(logits_bar, z):
    """Clipped double-Q in categorical form: per row, the target twin whose expected
    value sum_j softmax(l_i)_j z_j is the smaller (twin 0 on ties) supplies the whole
    distribution.  Returns (probabilities [n, N], chosen twin index [n])."""
    p0, p1 = softmax(logits_bar[0]), softmax(logits_bar[1])
    pick = (p1 @ z) < (p0 @ z)
    return np.where(pick[:, None], p1, p0), pick.astype(np.int64)


def mse_loss(q, y):
    """Eq. (2) for both twins: sum over twins of the batch mean of (Q_i - y)^2.
    q [2, n], y [n].  Returns (loss, dq) with dq = 2 (Q_i - y) / n."""
    n = y.shape[0]
    diff = q - y[None]
    return float(np.sum(np.mean(diff * diff, axis=1))), 2.0 * diff / n

