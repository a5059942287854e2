"""Independent torch (CPU, float64) re-statement of the agent's forward pass.

Used only to pin the oracle: torch's own conv2d / linear / layer_norm /
log_softmax and autograd differentiate this graph, so the oracle's
hand-written backward is checked against derivatives it did not compute.
"""
import math

import torch
import torch.nn.functional as F


def views(flat, table):
    return {n: flat[o:o + math.prod(s)].view(*s) for n, (o, s) in table.items()}


def encoder(P, x, n_conv):
    h = x
    for i in range(n_conv):
        h = F.relu(F.conv2d(h, P[f"enc.conv{i + 1}.W"], P[f"enc.conv{i + 1}.b"], stride=2 if i == 0 else 1))
    return h.flatten(1)


def dense(P, pre, x, act):
    y = F.layer_norm(F.linear(x, P[pre + ".W"], P[pre + ".b"]), (P[pre + ".W"].shape[0],),
                     P[pre + ".ln.g"], P[pre + ".ln.b"], eps=1e-5)
    return torch.tanh(y) if act == "tanh" else F.relu(y)


def critic(P, f, s, a):
    h = dense(P, "critic.trunk", f, "tanh")
    X = torch.cat([h, s, a], 1)
    out = []
    for q in ("q1", "q2"):
        g = dense(P, q + ".l2", dense(P, q + ".l1", X, "relu"), "relu")
        out.append(F.linear(g, P[q + ".out.W"], P[q + ".out.b"]))
    return torch.stack(out)


def actor(P, f, s, eps, lo, hi):
    h = dense(P, "actor.trunk", f, "tanh")
    g = dense(P, "actor.l2", dense(P, "actor.l1", torch.cat([h, s], 1), "relu"), "relu")
    out = F.linear(g, P["actor.out.W"], P["actor.out.b"])
    A = out.shape[1] // 2
    mu, us = out[:, :A], out[:, A:]
    log_std = lo + 0.5 * (hi - lo) * (torch.tanh(us) + 1)
    std = log_std.exp()
    u = mu + std * eps
    a = torch.tanh(u)
    # log density via torch.distributions, Jacobian via log1p(-tanh^2)
    lp = torch.distributions.Normal(mu, std).log_prob(u) - torch.log1p(-a * a)
    return a, lp.sum(1)


def rounding(on):
    """Operand rounding used by the bfloat16-operand mode, via torch's own cast."""
    if not on:
        return lambda t: t
    return lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def critic_bf16_fwd(P, f, s, a):
    """critic() with every GEMM operand cast to bfloat16 (forward only)."""
    r = rounding(True)

    def dn(pre, x, act):
        y = F.layer_norm(F.linear(r(x), r(P[pre + ".W"]), P[pre + ".b"]), (P[pre + ".W"].shape[0],),
                         P[pre + ".ln.g"], P[pre + ".ln.b"], eps=1e-5)
        return torch.tanh(y) if act == "tanh" else F.relu(y)
    h = dn("critic.trunk", f, "tanh")
    X = torch.cat([h, s, a], 1)
    out = []
    for q in ("q1", "q2"):
        g = dn(q + ".l2", dn(q + ".l1", X, "relu"), "relu")
        out.append(F.linear(r(g), r(P[q + ".out.W"]), P[q + ".out.b"]))
    return torch.stack(out)
