"""Network dimensions and the canonical flat parameter layout.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Architecture (Sec. IV, Encoder Design Choices and Normalization; Alg. 1):
a shared conv encoder (3x3 valid convolutions, the first with stride 2, each
followed by ReLU) feeds two separate one-layer projections, one for the
critics and one for the actor (Linear -> LayerNorm -> tanh).  The critic
projection is shared by the twin critics and is part of the EMA target.
Each twin critic is Linear -> LN -> ReLU -> Linear -> LN -> ReLU -> Linear to
`atoms` logits (C51, Sec. IV Critic Design Choices) on [h_c; proprio; action];
the actor is the same MLP on [h_a; proprio] with a 2*action output
(mean, pre-squash log-std).  The output heads carry no LayerNorm.

Flat order (every side builds it independently from this list):
  enc.conv{1..n}.{W[F,Cin,3,3], b[F]}
  critic.trunk.{W[proj,flat], b, ln.g, ln.b}
  q1.{l1.W[hid, proj+P+A], l1.b, l1.ln.g, l1.ln.b, l2.W[hid,hid], l2.b, l2.ln.g, l2.ln.b,
      out.W[atoms,hid], out.b}
  q2.(same as q1)
  actor.trunk.(same shapes as critic.trunk)
  actor.{l1.W[hid, proj+P], ..., out.W[2A,hid], out.b}
  log_alpha[1]
The target critic is a copy of the block critic.trunk .. q2.
"""
from collections import OrderedDict
from types import SimpleNamespace

TINY = dict(C=3, H=32, W=32, k=2, n_conv=2, F=16, proj=64, hidden=64, atoms=51,
            proprio=12, action=6, v_min=-10.0, v_max=10.0)
FULL = dict(C=9, H=64, W=64, k=4, n_conv=3, F=32, proj=256, hidden=512, atoms=101,
            proprio=12, action=6, v_min=-20.0, v_max=20.0)
FULL128 = dict(FULL, H=128, W=128, k=8)


def dims(**kw):
    d = SimpleNamespace(**kw)
    if d.n_conv == 0:
        # state-based SAC: no image and no encoder; the proprio state vector is
        # the feature that the projections read
        d.side, d.conv_sides, d.flat = 0, [], d.proprio
        d.critic_in = d.proj + d.proprio + d.action
        d.actor_in = d.proj + d.proprio
        return d
    d.side = d.H // d.k
    s = (d.side - 3) // 2 + 1
    d.conv_sides = [s]
    for _ in range(d.n_conv - 1):
        s = s - 2
        d.conv_sides.append(s)
    d.flat = d.F * s * s
    d.critic_in = d.proj + d.proprio + d.action
    d.actor_in = d.proj + d.proprio
    return d


def _trunk(prefix, d, out):
    out[prefix + ".W"] = (d.proj, d.flat)
    out[prefix + ".b"] = (d.proj,)
    out[prefix + ".ln.g"] = (d.proj,)
    out[prefix + ".ln.b"] = (d.proj,)


def _mlp(prefix, d, nin, nout, out):
    h = d.hidden
    out[prefix + ".l1.W"] = (h, nin)
    out[prefix + ".l1.b"] = (h,)
    out[prefix + ".l1.ln.g"] = (h,)
    out[prefix + ".l1.ln.b"] = (h,)
    out[prefix + ".l2.W"] = (h, h)
    out[prefix + ".l2.b"] = (h,)
    out[prefix + ".l2.ln.g"] = (h,)
    out[prefix + ".l2.ln.b"] = (h,)
    out[prefix + ".out.W"] = (nout, h)
    out[prefix + ".out.b"] = (nout,)


def shapes(d):
    out = OrderedDict()
    cin = d.C
    for i in range(d.n_conv):
        out[f"enc.conv{i + 1}.W"] = (d.F, cin, 3, 3)
        out[f"enc.conv{i + 1}.b"] = (d.F,)
        cin = d.F
    _trunk("critic.trunk", d, out)
    _mlp("q1", d, d.critic_in, d.atoms, out)
    _mlp("q2", d, d.critic_in, d.atoms, out)
    _trunk("actor.trunk", d, out)
    _mlp("actor", d, d.actor_in, 2 * d.action, out)
    out["log_alpha"] = (1,)
    return out


def _size(shape):
    n = 1
    for s in shape:
        n *= s
    return n


def offsets(d):
    """name -> (offset, shape) in the flat vector, plus the block boundaries."""
    off = 0
    table = OrderedDict()
    for name, shp in shapes(d).items():
        table[name] = (off, shp)
        off += _size(shp)
    return table, off


def blocks(d):
    """[start, end) of the encoder, critic (= target) and actor blocks."""
    table, total = offsets(d)
    enc_end = table["critic.trunk.W"][0]
    critic_end = table["actor.trunk.W"][0]
    actor_end = table["log_alpha"][0]
    return dict(enc=(0, enc_end), critic=(enc_end, critic_end),
                actor=(critic_end, actor_end), log_alpha=(actor_end, total), total=total)


def view(flat, d, prefix=""):
    """Dict of reshaped views into a flat parameter vector."""
    table, _ = offsets(d)
    return {n: flat[o:o + _size(s)].reshape(s) for n, (o, s) in table.items()
            if n.startswith(prefix)}


def target_view(target_flat, d):
    """Views of the target critic vector (a copy of the critic block)."""
    table, _ = offsets(d)
    base = blocks(d)["critic"][0]
    out = {}
    for n, (o, s) in table.items():
        if n.startswith(("critic.", "q1.", "q2.")):
            out[n] = target_flat[o - base:o - base + _size(s)].reshape(s)
    return out
