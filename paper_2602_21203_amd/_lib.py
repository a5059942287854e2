"""ctypes binding of libsquint (include/squint.h): argument marshalling only.

Every computation runs in the library's HIP kernels; torch tensors only supply
device memory and the current stream.  Importing this module loads the shared
library and fails loudly if it has not been built.
"""
import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SQ_LIB_PATH") or os.path.join(HERE, "libsquint.so")

SQ_OK, SQ_EINVAL, SQ_ENOMEM, SQ_EDEVICE, SQ_ECAPTURE = 0, 1, 2, 3, 4
SQ_F32, SQ_BF16 = 0, 1
SQ_OP_ENCODER, SQ_OP_CRITIC, SQ_OP_ACTOR = 0, 1, 2
N_STATS = 8
STAT_NAMES = ("critic_loss", "actor_loss", "alpha_loss", "alpha", "entropy", "mean_q", "mean_target", "nonfinite")

c_int, c_float, c_ll, c_ull, c_vp, c_size = (ctypes.c_int, ctypes.c_float, ctypes.c_longlong,
                                             ctypes.c_ulonglong, ctypes.c_void_p, ctypes.c_size_t)


class Dims(ctypes.Structure):
    _fields_ = [(n, c_int) for n in ("C", "H", "W", "k", "n_conv", "F", "proj", "hidden", "atoms",
                                     "proprio", "action")] + [("v_min", c_float), ("v_max", c_float)]


class HParams(ctypes.Structure):
    _fields_ = [(n, c_float) for n in ("gamma", "lr", "beta1", "beta2", "adam_eps", "rho", "target_entropy",
                                       "log_std_min", "log_std_max")] + \
               [("policy_freq", c_int), ("prec", c_int), ("seed", c_ull), ("cdq", c_int)]


class Replay(ctypes.Structure):
    _fields_ = [(n, c_vp) for n in ("obs", "next_obs", "proprio", "next_proprio", "action", "reward", "done")] + \
               [("capacity", c_int), ("size", c_int), ("squinted", c_int), ("dev_size", c_vp)]


class EnvBuffers(ctypes.Structure):
    _fields_ = [("obs", c_vp * 2), ("proprio", c_vp), ("next_obs", c_vp), ("proprio_t", c_vp),
                ("next_proprio", c_vp), ("reward", c_vp), ("done", c_vp)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", c_ll), ("requests", c_ll), ("rows", c_ll), ("fused_batches", c_ll),
                ("max_requests_per_batch", c_int), ("max_slots_busy", c_int), ("overlapped_batches", c_ll),
                ("device_busy_s", ctypes.c_double), ("device_span_s", ctypes.c_double)]


DONE_CB = ctypes.CFUNCTYPE(None, ctypes.c_ulonglong, ctypes.c_double, ctypes.c_void_p)


class SquintError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2602_21203_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "sq_last_error": (ctypes.c_char_p, []),
        "sq_version": (c_int, []),
        "sq_param_count": (c_int, [P(Dims), P(c_ll)]),
        "sq_param_tensor_count": (c_int, [P(Dims), P(c_int)]),
        "sq_param_offsets": (c_int, [P(Dims), P(c_ll), P(c_ll)]),
        "sq_workspace_bytes": (c_int, [P(Dims), c_int, c_int, P(c_size)]),
        "squint_downsample": (c_int, [P(Dims), c_vp, c_vp, c_int, c_int, c_vp, c_vp]),
        "encoder_fwd": (c_int, [P(Dims), c_int, c_vp, c_vp, c_int, c_vp, c_vp, c_vp]),
        "encoder_bwd": (c_int, [P(Dims), c_int, c_vp, c_vp, c_vp, c_int, c_vp, c_vp]),
        "critic_fwd": (c_int, [P(Dims), c_int, c_vp, c_vp, c_vp, c_vp, c_int, c_vp, c_vp, c_vp]),
        "critic_bwd": (c_int, [P(Dims), c_int, c_vp, c_vp, c_vp, c_int, c_vp, c_vp, c_vp, c_vp]),
        "c51_project": (c_int, [P(Dims), c_vp, c_vp, c_vp, c_vp, c_float, c_int, c_vp, c_vp]),
        "actor_fwd": (c_int, [P(Dims), c_int, P(HParams), c_vp, c_vp, c_vp, c_vp, c_int, c_vp, c_vp, c_vp, c_vp]),
        "actor_bwd": (c_int, [P(Dims), c_int, P(HParams), c_vp, c_vp, c_vp, c_vp, c_int, c_vp, c_vp]),
        "adam_step": (c_int, [c_vp, c_vp, c_vp, c_vp, c_ll, P(HParams), c_vp, c_vp, c_vp, c_ll, c_vp]),
        "sq_agent_create": (c_int, [P(Dims), P(HParams), c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, P(c_vp)]),
        "sq_agent_destroy": (c_int, [c_vp]),
        "sq_agent_sync": (c_int, [c_vp, c_vp]),
        "sac_update": (c_int, [c_vp, P(Replay), c_int, c_vp, c_vp]),
        "sac_update_eager": (c_int, [c_vp, P(Replay), c_int, c_vp, c_vp]),
        "act": (c_int, [c_vp, c_vp, c_vp, c_int, c_int, c_ull, c_vp, c_vp]),
        "sq_agent_act_capacity": (c_int, [c_vp, P(c_int)]),
        "sq_server_create": (c_int, [c_vp, c_size, c_int, c_int, P(c_vp)]),
        "sq_server_submit": (c_int, [c_vp, c_vp, c_vp, c_int, c_int, c_ull, c_vp, DONE_CB, c_vp]),
        "sq_server_drain": (c_int, [c_vp]),
        "sq_server_destroy": (c_int, [c_vp]),
        "sq_server_hold": (c_int, [c_vp, c_int]),
        "sq_server_get_stats": (c_int, [c_vp, P(ServerStats)]),
        "sq_ring_create": (c_int, [P(Dims), c_int, P(c_vp)]),
        "sq_ring_destroy": (c_int, [c_vp]),
        "sq_ring_insert": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_int, c_vp]),
        "sq_ring_view": (c_int, [c_vp, P(Replay)]),
        "sq_ring_state": (c_int, [c_vp, P(c_int), P(c_int)]),
        "sq_ring_copy_out": (c_int, [c_vp, c_int, c_int, c_int, c_vp, c_vp]),
        "sq_env_create": (c_int, [P(Dims), c_int, c_int, c_ull, P(EnvBuffers), P(c_vp)]),
        "sq_env_destroy": (c_int, [c_vp]),
        "sq_env_step": (c_int, [c_vp, c_vp, c_vp]),
        "sq_gemm": (c_int, [c_int, c_int, c_int, c_int, c_int, c_vp, c_ll, c_ll, c_ll, c_vp, c_ll, c_ll, c_ll,
                            c_vp, c_ll, c_ll, c_vp, c_ll, c_int, c_vp]),
        "sq_sample_indices": (c_int, [c_ull, ctypes.c_uint, c_int, c_int, c_vp, c_vp]),
        "sq_gaussian": (c_int, [c_ull, ctypes.c_uint, ctypes.c_uint, c_int, c_vp, c_vp]),
        "sq_agent_graph_count": (c_int, [c_vp, P(c_ll), P(c_int)]),
        "sq_agent_last_indices": (c_int, [c_vp, c_vp, c_vp]),
        "sq_agent_last_target": (c_int, [c_vp, c_vp, c_vp]),
        "sq_ring_row": (c_int, [c_int, c_ll, c_int, P(c_int)]),
        "sq_gemm_tile_order": (c_int, [c_int, c_int, c_int, c_int, P(c_int)]),
        "sq_bf16_operand_copies": (c_int, [c_int]),
        "sq_bf16_copy_products": (c_int, [P(c_ll)]),
        "sq_gemm_bf16": (c_int, [c_int, c_int, c_int, c_int, c_vp, c_ll, c_ll, c_ll, c_vp, c_ll, c_ll, c_ll, c_vp,
                                 c_ll, c_ll, c_vp, c_ll, c_vp]),
        "encoder_fwd_noalloc": (c_int, [P(Dims), c_int, c_vp, c_vp, c_int, c_vp, c_vp]),
        "sq_encoder_noalloc_max_images": (c_int, [P(Dims), P(c_int)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def check(status):
    if status != SQ_OK:
        msg = LIB.sq_last_error().decode(errors="replace")
        raise SquintError(f"libsquint status {status}: {msg}")


def ptr(t):
    """Device (or host) address of a tensor, None for None."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_dims(cfg):
    return Dims(cfg["C"], cfg["H"], cfg["W"], cfg["k"], cfg["n_conv"], cfg["F"], cfg["proj"], cfg["hidden"],
                cfg["atoms"], cfg["proprio"], cfg["action"], float(cfg["v_min"]), float(cfg["v_max"]))


def make_hparams(action, prec=SQ_F32, gamma=0.99, lr=3e-4, beta1=0.9, beta2=0.999, adam_eps=1e-8, rho=0.995,
                 target_entropy=None, log_std_min=-5.0, log_std_max=2.0, policy_freq=1, seed=2, cdq=False):
    te = -float(action) if target_entropy is None else target_entropy
    return HParams(gamma, lr, beta1, beta2, adam_eps, rho, te, log_std_min, log_std_max, policy_freq, prec, seed,
                   int(bool(cdq)))


# canonical tensor names, in library order (the shapes come from the dims)
def _names(n_conv):
    out = []
    for i in range(n_conv):
        out += [f"enc.conv{i + 1}.W", f"enc.conv{i + 1}.b"]
    dense = lambda p: [p + ".W", p + ".b", p + ".ln.g", p + ".ln.b"]
    mlp = lambda p: dense(p + ".l1") + dense(p + ".l2") + [p + ".out.W", p + ".out.b"]
    out += dense("critic.trunk") + mlp("q1") + mlp("q2") + dense("actor.trunk") + mlp("actor") + ["log_alpha"]
    return out


def _shapes(cfg):
    F, P, H, A, S = cfg["F"], cfg["proj"], cfg["hidden"], cfg["action"], cfg["proprio"]
    if cfg["n_conv"] == 0:          # state-based: the proprio state is the feature
        flat = S
    else:
        side = cfg["H"] // cfg["k"]
        s = (side - 3) // 2 + 1
        for _ in range(cfg["n_conv"] - 1):
            s -= 2
        flat = F * s * s
    shp = {}
    cin = cfg["C"]
    for i in range(cfg["n_conv"]):
        shp[f"enc.conv{i + 1}.W"] = (F, cin, 3, 3)
        shp[f"enc.conv{i + 1}.b"] = (F,)
        cin = F
    for pre, nin, nout in (("q1", P + S + A, cfg["atoms"]), ("q2", P + S + A, cfg["atoms"]), ("actor", P + S, 2 * A)):
        shp.update({pre + ".l1.W": (H, nin), pre + ".l2.W": (H, H), pre + ".out.W": (nout, H), pre + ".out.b": (nout,)})
        for l in ("l1", "l2"):
            for t in ("b", "ln.g", "ln.b"):
                shp[f"{pre}.{l}.{t}"] = (H,)
    for pre in ("critic.trunk", "actor.trunk"):
        shp[pre + ".W"] = (P, flat)
        for t in ("b", "ln.g", "ln.b"):
            shp[f"{pre}.{t}"] = (P,)
    shp["log_alpha"] = (1,)
    return shp, flat


def param_table(cfg):
    """[(name, offset, shape)] from the library's offsets, checked against the shapes."""
    d = make_dims(cfg)
    cnt = c_int()
    check(LIB.sq_param_tensor_count(ctypes.byref(d), ctypes.byref(cnt)))
    off = (c_ll * (cnt.value + 1))()
    blocks = (c_ll * 4)()
    check(LIB.sq_param_offsets(ctypes.byref(d), off, blocks))
    names = _names(cfg["n_conv"])
    shapes, _ = _shapes(cfg)
    assert len(names) == cnt.value
    table = []
    for i, n in enumerate(names):
        size = off[i + 1] - off[i]
        assert size == math.prod(shapes[n]), (n, size, shapes[n])
        table.append((n, int(off[i]), shapes[n]))
    return table, dict(enc=(0, int(blocks[1])), critic=(int(blocks[1]), int(blocks[2])),
                       actor=(int(blocks[2]), int(blocks[3])), log_alpha=(int(blocks[3]), int(off[cnt.value])),
                       total=int(off[cnt.value]))


def param_count(cfg):
    n = c_ll()
    check(LIB.sq_param_count(ctypes.byref(make_dims(cfg)), ctypes.byref(n)))
    return n.value


def workspace_bytes(cfg, op, n):
    b = c_size()
    check(LIB.sq_workspace_bytes(ctypes.byref(make_dims(cfg)), op, n, ctypes.byref(b)))
    return b.value


def feat_width(cfg):
    return _shapes(cfg)[1]
