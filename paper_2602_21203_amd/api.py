"""Python face of libsquint: the C entry points under the same names, taking
torch tensors.  Marshalling only -- shapes are checked on the host, outputs are
allocated with torch, and every step runs in the library's kernels on the
current HIP stream.
"""
import ctypes

import torch

from . import _lib as L
from ._lib import SQ_BF16, SQ_F32, check, ptr, stream_handle


def _dims(cfg):
    return ctypes.byref(L.make_dims(cfg))


def _req(t, dtype, shape=None, name="tensor"):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _side(cfg):
    return cfg["H"] // cfg["k"]


def squint_downsample(cfg, frames, idx=None, n=None, prec=SQ_F32, out=None, stream=None):
    """[rows, H, W, C] uint8 (+ optional idx [n] int32) -> [n, C, 16, 16] f32 or bf16."""
    _req(frames, torch.uint8, name="frames")
    if frames.dim() != 4 or tuple(frames.shape[1:]) != (cfg["H"], cfg["W"], cfg["C"]):
        raise ValueError(f"frames shape {tuple(frames.shape)} does not match the dims")
    if idx is not None:
        _req(idx, torch.int32, name="idx")
        n = idx.numel() if n is None else n
    n = frames.shape[0] if n is None else n
    s = _side(cfg)
    dt = torch.float32 if prec == SQ_F32 else torch.bfloat16
    if out is None:
        out = torch.empty((n, cfg["C"], s, s), dtype=dt, device=frames.device)
    _req(out, dt, (n, cfg["C"], s, s), "out")
    check(L.LIB.squint_downsample(_dims(cfg), ptr(frames), ptr(idx), n, prec, ptr(out), stream_handle(stream)))
    return out


def encoder_fwd(cfg, prec, enc_params, x, ws=None, stream=None):
    n = x.shape[0]
    s = _side(cfg)
    _req(x, torch.float32, (n, cfg["C"], s, s), "x")
    _req(enc_params, torch.float32, name="enc_params")
    if ws is None:
        ws = torch.empty(L.workspace_bytes(cfg, L.SQ_OP_ENCODER, n), dtype=torch.uint8, device=x.device)
    feat = torch.empty((n, L.feat_width(cfg)), dtype=torch.float32, device=x.device)
    check(L.LIB.encoder_fwd(_dims(cfg), prec, ptr(enc_params), ptr(x), n, ptr(feat), ptr(ws), stream_handle(stream)))
    return feat, ws


def encoder_fwd_noalloc(cfg, prec, enc_params, x, feat=None, stream=None):
    """encoder_fwd with the library's fixed scratch instead of a workspace."""
    n = x.shape[0]
    s = _side(cfg)
    _req(x, torch.float32, (n, cfg["C"], s, s), "x")
    _req(enc_params, torch.float32, name="enc_params")
    if feat is None:
        feat = torch.empty((n, L.feat_width(cfg)), dtype=torch.float32, device=x.device)
    _req(feat, torch.float32, (n, L.feat_width(cfg)), "feat")
    check(L.LIB.encoder_fwd_noalloc(_dims(cfg), prec, ptr(enc_params), ptr(x), n, ptr(feat), stream_handle(stream)))
    return feat


def encoder_noalloc_max_images(cfg):
    n = ctypes.c_int()
    check(L.LIB.sq_encoder_noalloc_max_images(_dims(cfg), ctypes.byref(n)))
    return n.value


def encoder_bwd(cfg, prec, enc_params, ws, dfeat, n_enc_params, stream=None):
    n = dfeat.shape[0]
    _req(dfeat, torch.float32, (n, L.feat_width(cfg)), "dfeat")
    d = torch.empty(n_enc_params, dtype=torch.float32, device=dfeat.device)
    check(L.LIB.encoder_bwd(_dims(cfg), prec, ptr(enc_params), ptr(ws), ptr(dfeat), n, ptr(d), stream_handle(stream)))
    return d


def critic_fwd(cfg, prec, critic_params, feat, proprio, action, ws=None, stream=None):
    n = feat.shape[0]
    _req(feat, torch.float32, (n, L.feat_width(cfg)), "feat")
    _req(proprio, torch.float32, (n, cfg["proprio"]), "proprio")
    _req(action, torch.float32, (n, cfg["action"]), "action")
    _req(critic_params, torch.float32, name="critic_params")
    if ws is None:
        ws = torch.empty(L.workspace_bytes(cfg, L.SQ_OP_CRITIC, n), dtype=torch.uint8, device=feat.device)
    logits = torch.empty((2, n, cfg["atoms"]), dtype=torch.float32, device=feat.device)
    check(L.LIB.critic_fwd(_dims(cfg), prec, ptr(critic_params), ptr(feat), ptr(proprio), ptr(action), n, ptr(logits),
                           ptr(ws), stream_handle(stream)))
    return logits, ws


def critic_bwd(cfg, prec, critic_params, ws, dlogits, want_params=True, want_feat=True, want_action=True,
               stream=None):
    n = dlogits.shape[1]
    _req(dlogits, torch.float32, (2, n, cfg["atoms"]), "dlogits")
    dev = dlogits.device
    dp = torch.empty_like(critic_params) if want_params else None
    df = torch.empty((n, L.feat_width(cfg)), dtype=torch.float32, device=dev) if want_feat else None
    da = torch.empty((n, cfg["action"]), dtype=torch.float32, device=dev) if want_action else None
    check(L.LIB.critic_bwd(_dims(cfg), prec, ptr(critic_params), ptr(ws), ptr(dlogits), n, ptr(dp), ptr(df), ptr(da),
                           stream_handle(stream)))
    return dp, df, da


def c51_project(cfg, p_next, reward, done, bonus, gamma, stream=None):
    n = p_next.shape[0]
    _req(p_next, torch.float32, (n, cfg["atoms"]), "p_next")
    _req(reward, torch.float32, (n,), "reward")
    _req(done, torch.uint8, (n,), "done")
    if bonus is not None:
        _req(bonus, torch.float32, (n,), "bonus")
    m = torch.empty_like(p_next)
    check(L.LIB.c51_project(_dims(cfg), ptr(p_next), ptr(reward), ptr(done), ptr(bonus), float(gamma), n, ptr(m),
                            stream_handle(stream)))
    return m


def actor_fwd(cfg, prec, hp, actor_params, feat, proprio, eps=None, ws=None, stream=None):
    n = feat.shape[0]
    _req(feat, torch.float32, (n, L.feat_width(cfg)), "feat")
    _req(proprio, torch.float32, (n, cfg["proprio"]), "proprio")
    if eps is not None:
        _req(eps, torch.float32, (n, cfg["action"]), "eps")
    if ws is None:
        ws = torch.empty(L.workspace_bytes(cfg, L.SQ_OP_ACTOR, n), dtype=torch.uint8, device=feat.device)
    action = torch.empty((n, cfg["action"]), dtype=torch.float32, device=feat.device)
    logp = torch.empty((n,), dtype=torch.float32, device=feat.device) if eps is not None else None
    check(L.LIB.actor_fwd(_dims(cfg), prec, ctypes.byref(hp), ptr(actor_params), ptr(feat), ptr(proprio), ptr(eps), n,
                          ptr(action), ptr(logp), ptr(ws), stream_handle(stream)))
    return action, logp, ws


def actor_bwd(cfg, prec, hp, actor_params, ws, daction, dlogp, stream=None):
    n = daction.shape[0]
    _req(daction, torch.float32, (n, cfg["action"]), "daction")
    if dlogp is not None:
        _req(dlogp, torch.float32, (n,), "dlogp")
    dp = torch.empty_like(actor_params)
    check(L.LIB.actor_bwd(_dims(cfg), prec, ctypes.byref(hp), ptr(actor_params), ptr(ws), ptr(daction), ptr(dlogp), n,
                          ptr(dp), stream_handle(stream)))
    return dp


def adam_step(p, g, m, v, hp, step, p_bf16=None, ema_target=None, ema_begin=0, stream=None):
    n = p.numel()
    for t, nm in ((p, "p"), (g, "g"), (m, "m"), (v, "v")):
        _req(t, torch.float32, (n,), nm)
    _req(step, torch.int32, name="step")
    check(L.LIB.adam_step(ptr(p), ptr(g), ptr(m), ptr(v), n, ctypes.byref(hp), ptr(step), ptr(p_bf16), ptr(ema_target),
                          int(ema_begin), stream_handle(stream)))


def gemm(prec, A, B, C=None, bias=None, accumulate=False, transpose_b=True, stream=None):
    """C[z] = A[z] @ op(B[z]) (+ bias), op(B) = B^T (B given as [N, K]) or B ([K, N]).

    A: [batch, M, K] or [M, K]; strides are passed through, so views work."""
    a3 = A if A.dim() == 3 else A.unsqueeze(0)
    b3 = B if B.dim() == 3 else B.unsqueeze(0)
    batch, M, K = a3.shape
    N = b3.shape[1] if transpose_b else b3.shape[2]
    if C is None:
        C = torch.zeros((batch, M, N), dtype=torch.float32, device=A.device)
    c3 = C if C.dim() == 3 else C.unsqueeze(0)
    for t in (a3, b3, c3):
        if t.dtype != torch.float32 or not t.is_cuda:
            raise ValueError("gemm takes float32 device tensors")
    b_lr, b_lk = (b3.stride(1), b3.stride(2)) if transpose_b else (b3.stride(2), b3.stride(1))
    if c3.stride(2) != 1:
        raise ValueError("C must be row-major")
    bz = b3.stride(0) if b3.shape[0] > 1 else 0
    bias_sz = 0
    if bias is not None:
        bias_sz = bias.stride(0) if bias.dim() == 2 and bias.shape[0] > 1 else 0
    check(L.LIB.sq_gemm(prec, M, N, K, batch, ptr(a3), a3.stride(1), a3.stride(2), a3.stride(0) if batch > 1 else 0,
                        ptr(b3), b_lr, b_lk, bz, ptr(c3), c3.stride(1), c3.stride(0) if batch > 1 else 0, ptr(bias),
                        bias_sz, int(bool(accumulate)), stream_handle(stream)))
    return C


def _bf16_operand(t, name):
    """(tensor [batch, rows, K], lr, lk, sz) of a bfloat16 operand: k-contiguous rows
    holding K rounded up to 8, or contiguous rows (k strided) with k-slices holding
    the row count rounded up to 8; 16-byte aligned."""
    t3 = t if t.dim() == 3 else t.unsqueeze(0)
    if t3.dtype != torch.bfloat16 or not t3.is_cuda:
        raise ValueError(f"{name}: bfloat16 device tensor expected")
    batch, rows, K = t3.shape
    lr, lk, sz = t3.stride(1), t3.stride(2), (t3.stride(0) if batch > 1 else 0)
    r8 = lambda x: (x + 7) // 8 * 8
    if lk == 1:
        ld, n_lines, length = lr, rows, r8(K)
    elif lr == 1:
        ld, n_lines, length = lk, K, r8(rows)
    else:
        raise ValueError(f"{name}: k-contiguous rows or contiguous rows expected")
    need = t3.storage_offset() + (batch - 1) * sz + (n_lines - 1) * ld + length
    if ld % 8 or sz % 8 or ld < length or t3.data_ptr() % 16 or need > t3.untyped_storage().nbytes() // 2:
        raise ValueError(f"{name}: lines must be 16-byte aligned and hold their length rounded up to 8 elements")
    return t3, lr, lk, sz


def gemm_bf16(A, B, C=None, bias=None, stream=None):
    """C[z] = A[z] @ B[z]^T (+ bias) on bfloat16 operands (A [batch, M, K], B [batch, N, K];
    each k-contiguous, or transposed with contiguous rows): the kernel of the products
    that read bfloat16 copies, equal to gemm(SQ_BF16, ...) on the FP32 values of A and B."""
    a3, a_lr, a_lk, a_sz = _bf16_operand(A, "A")
    b3, b_lr, b_lk, b_sz = _bf16_operand(B, "B")
    batch, M, K = a3.shape
    N = b3.shape[1]
    if b3.shape[2] != K or b3.shape[0] not in (1, batch):
        raise ValueError("A and B disagree in K or batch")
    if C is None:
        C = torch.zeros((batch, M, N), dtype=torch.float32, device=A.device)
    c3 = C if C.dim() == 3 else C.unsqueeze(0)
    if c3.dtype != torch.float32 or c3.stride(2) != 1:
        raise ValueError("C must be a row-major float32 tensor")
    bias_sz = 0
    if bias is not None:
        bias_sz = bias.stride(0) if bias.dim() == 2 and bias.shape[0] > 1 else 0
    check(L.LIB.sq_gemm_bf16(M, N, K, batch, ptr(a3), a_lr, a_lk, a_sz, ptr(b3), b_lr, b_lk,
                             b_sz if b3.shape[0] > 1 else 0, ptr(c3), c3.stride(1), c3.stride(0) if batch > 1 else 0,
                             ptr(bias), bias_sz, stream_handle(stream)))
    return C


def bf16_operand_copies(on):
    """Whether agents created from now on in the bfloat16 mode keep bfloat16 copies of
    their products' operands (the default); returns the previous setting."""
    return bool(L.LIB.sq_bf16_operand_copies(int(bool(on))))


def bf16_copy_products():
    """Linear-layer products enqueued on bfloat16 copies so far in this process."""
    n = ctypes.c_longlong()
    check(L.LIB.sq_bf16_copy_products(ctypes.byref(n)))
    return n.value


def sample_indices(seed, update, size, n, device="cuda", stream=None):
    idx = torch.empty(n, dtype=torch.int32, device=device)
    check(L.LIB.sq_sample_indices(seed, update, size, n, ptr(idx), stream_handle(stream)))
    return idx


def gaussian(seed, update, stream_id, n, device="cuda", stream=None):
    e = torch.empty(n, dtype=torch.float32, device=device)
    check(L.LIB.sq_gaussian(seed, update, stream_id, n, ptr(e), stream_handle(stream)))
    return e


def replay_struct(rep):
    """sq_replay view of a dict of device tensors (synthetic.replay layout)."""
    cap = rep["obs"].shape[0]
    for k, dt in (("obs", torch.uint8), ("next_obs", torch.uint8), ("proprio", torch.float32),
                  ("next_proprio", torch.float32), ("action", torch.float32), ("reward", torch.float32),
                  ("done", torch.uint8)):
        _req(rep[k], dt, name=k)
        if rep[k].shape[0] != cap:
            raise ValueError(f"replay field {k} has {rep[k].shape[0]} rows, expected {cap}")
    return L.Replay(*(ptr(rep[k]) for k in ("obs", "next_obs", "proprio", "next_proprio", "action", "reward",
                                            "done")), cap, int(rep.get("size", cap)))


class Ring:
    """Device FIFO replay of transitions squinted at insertion (library-owned rows).

    insert() squints raw [n, H, W, C] uint8 frames into uint8 block means and
    appends the transitions; view is the sq_replay that Agent.sac_update samples."""

    def __init__(self, cfg, capacity):
        self.cfg = cfg
        self.capacity = int(capacity)
        h = ctypes.c_void_p()
        check(L.LIB.sq_ring_create(_dims(cfg), self.capacity, ctypes.byref(h)))
        self.handle = h
        self.view = L.Replay()
        check(L.LIB.sq_ring_view(self.handle, ctypes.byref(self.view)))
        side = cfg["H"] // cfg["k"]
        self.frame_shape = (side, side, cfg["C"])

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            L.LIB.sq_ring_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, obs, next_obs, proprio, next_proprio, action, reward, done, stream=None):
        n = obs.shape[0]
        c = self.cfg
        _req(obs, torch.uint8, (n, c["H"], c["W"], c["C"]), "obs")
        _req(next_obs, torch.uint8, (n, c["H"], c["W"], c["C"]), "next_obs")
        _req(proprio, torch.float32, (n, c["proprio"]), "proprio")
        _req(next_proprio, torch.float32, (n, c["proprio"]), "next_proprio")
        _req(action, torch.float32, (n, c["action"]), "action")
        _req(reward, torch.float32, (n,), "reward")
        _req(done, torch.uint8, (n,), "done")
        check(L.LIB.sq_ring_insert(self.handle, ptr(obs), ptr(next_obs), ptr(proprio), ptr(next_proprio),
                                   ptr(action), ptr(reward), ptr(done), n, stream_handle(stream)))

    FIELDS = ("obs", "next_obs", "proprio", "next_proprio", "action", "reward", "done")

    def read(self, field, row0=0, n=None, stream=None):
        """Rows [row0, row0 + n) of one stored field as a new device tensor."""
        n = self.capacity - row0 if n is None else n
        c = self.cfg
        shape, dt = {"obs": ((n,) + self.frame_shape, torch.uint8), "next_obs": ((n,) + self.frame_shape, torch.uint8),
                     "proprio": ((n, c["proprio"]), torch.float32), "next_proprio": ((n, c["proprio"]), torch.float32),
                     "action": ((n, c["action"]), torch.float32), "reward": ((n,), torch.float32),
                     "done": ((n,), torch.uint8)}[field]
        out = torch.empty(shape, dtype=dt, device="cuda")
        check(L.LIB.sq_ring_copy_out(self.handle, self.FIELDS.index(field), row0, n, ptr(out), stream_handle(stream)))
        return out

    def state(self):
        pos, size = ctypes.c_int(), ctypes.c_int()
        check(L.LIB.sq_ring_state(self.handle, ctypes.byref(pos), ctypes.byref(size)))
        return pos.value, size.value


class Env:
    """The synthetic environment stub (point mass, integer frame renderer) over
    torch-owned device buffers.  obs / proprio are the current observation;
    transition() gives the last step's transition as tensors (valid until the
    next step)."""

    def __init__(self, cfg, n_envs, episode_len=50, seed=3, device="cuda"):
        self.cfg, self.n = cfg, int(n_envs)
        frame = (self.n, cfg["H"], cfg["W"], cfg["C"])
        u8, f32 = dict(dtype=torch.uint8, device=device), dict(dtype=torch.float32, device=device)
        self.obs_buf = [torch.zeros(frame, **u8), torch.zeros(frame, **u8)]
        self.proprio = torch.zeros((self.n, cfg["proprio"]), **f32)
        self.next_obs = torch.zeros(frame, **u8)
        self.proprio_t = torch.zeros((self.n, cfg["proprio"]), **f32)
        self.next_proprio = torch.zeros((self.n, cfg["proprio"]), **f32)
        self.reward = torch.zeros(self.n, **f32)
        self.done = torch.zeros(self.n, **u8)
        self.action = None
        self.cur = 0
        bufs = L.EnvBuffers((ctypes.c_void_p * 2)(self.obs_buf[0].data_ptr(), self.obs_buf[1].data_ptr()),
                            self.proprio.data_ptr(), self.next_obs.data_ptr(), self.proprio_t.data_ptr(),
                            self.next_proprio.data_ptr(), self.reward.data_ptr(), self.done.data_ptr())
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        check(L.LIB.sq_env_create(_dims(cfg), self.n, int(episode_len), int(seed), ctypes.byref(bufs),
                                  ctypes.byref(h)))
        self.handle = h

    @property
    def obs(self):
        return self.obs_buf[self.cur]

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            L.LIB.sq_env_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, action, stream=None):
        _req(action, torch.float32, (self.n, self.cfg["action"]), "action")
        check(L.LIB.sq_env_step(self.handle, ptr(action), stream_handle(stream)))
        self.action = action
        self.cur ^= 1

    def transition(self):
        """(obs, next_obs, proprio, next_proprio, action, reward, done) of the last step."""
        return (self.obs_buf[self.cur ^ 1], self.next_obs, self.proprio_t, self.next_proprio, self.action,
                self.reward, self.done)


class Agent:
    """Owns the state tensors of one agent and the library handle.

    params: flat FP32 vector in the library's layout; the target starts as a
    copy of the critic block, moments and counters at zero."""

    def __init__(self, cfg, params, batch, prec=SQ_F32, device="cuda", **hp_kw):
        self.cfg = cfg
        self.table, self.blocks = L.param_table(cfg)
        self.batch = batch
        self.hp = L.make_hparams(cfg["action"], prec=prec, **hp_kw)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(device).contiguous()
        if self.params.numel() != self.blocks["total"]:
            raise ValueError("params has the wrong length")
        c0, c1 = self.blocks["critic"]
        self.target = self.params[c0:c1].clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.counters = torch.zeros(4, dtype=torch.int32, device=device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        check(L.LIB.sq_agent_create(_dims(cfg), ctypes.byref(self.hp), batch, ptr(self.params), ptr(self.target),
                                    ptr(self.m), ptr(self.v), ptr(self.grads), ptr(self.counters), ctypes.byref(h)))
        self.handle = h
        # graphs cannot be captured on the null stream: updates run on a side
        # stream ordered against the caller's current stream
        self.stream = torch.cuda.Stream(device=self.params.device)

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            L.LIB.sq_agent_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sac_update(self, replay, n_updates, stats=None, graph=True, stream=None):
        """replay: a dict of device tensors (raw frames) or a Ring."""
        # the view is rebuilt on every call (a few pointers), so a dict whose
        # size grew or whose tensors were replaced is seen as it is now
        rs = replay.view if isinstance(replay, Ring) else replay_struct(replay)
        if stats is None:
            stats = torch.empty((n_updates, L.N_STATS), dtype=torch.float32, device=self.params.device)
        _req(stats, torch.float32, (n_updates, L.N_STATS), "stats")
        fn = L.LIB.sac_update if graph else L.LIB.sac_update_eager
        caller = stream if stream is not None else torch.cuda.current_stream()
        # a caller already on the agent's stream is ordered by the stream itself;
        # any other stream is joined both ways (each join costs a cross-stream
        # wait on the device, so loops should pass stream=agent.stream)
        joined = caller.cuda_stream != self.stream.cuda_stream
        if joined:
            self.stream.wait_stream(caller)
        check(fn(self.handle, ctypes.byref(rs), n_updates, ptr(stats), stream_handle(self.stream)))
        if joined:
            caller.wait_stream(self.stream)
        return stats

    def graph_count(self):
        """(graphs captured so far, graphs cached) by sac_update."""
        n, c = ctypes.c_longlong(), ctypes.c_int()
        check(L.LIB.sq_agent_graph_count(self.handle, ctypes.byref(n), ctypes.byref(c)))
        return n.value, c.value

    def last_indices(self, stream=None):
        """Replay rows drawn by the last enqueued update ([batch] int32, device),
        ordered after it on the agent's stream."""
        idx = torch.empty(self.batch, dtype=torch.int32, device=self.params.device)
        st = self.stream if stream is None else stream
        check(L.LIB.sq_agent_last_indices(self.handle, ptr(idx), stream_handle(st)))
        st.synchronize()
        return idx

    def last_target(self, stream=None):
        """Projected target distribution m of the last enqueued update ([batch,
        atoms] float32, device; C51 heads only), ordered after it on the agent's
        stream."""
        m = torch.empty((self.batch, self.cfg["atoms"]), dtype=torch.float32, device=self.params.device)
        st = self.stream if stream is None else stream
        check(L.LIB.sq_agent_last_target(self.handle, ptr(m), stream_handle(st)))
        st.synchronize()
        return m

    def sync(self, stream=None):
        """Refresh the agent's derived weight copies after params / target were
        changed from outside (sq_agent_sync)."""
        check(L.LIB.sq_agent_sync(self.handle, stream_handle(stream)))

    def act(self, frames, proprio, sample=False, request_id=0, out=None, stream=None):
        n = frames.shape[0]
        _req(frames, torch.uint8, (n, self.cfg["H"], self.cfg["W"], self.cfg["C"]), "frames")
        _req(proprio, torch.float32, (n, self.cfg["proprio"]), "proprio")
        if out is None:
            out = torch.empty((n, self.cfg["action"]), dtype=torch.float32, device=frames.device)
        check(L.LIB.act(self.handle, ptr(frames), ptr(proprio), n, int(bool(sample)), int(request_id), ptr(out),
                        stream_handle(stream)))
        return out


class Server:
    """Continuous-batching act() server over an Agent's resident weights.

    submit() enqueues a request (its buffers must stay alive until done);
    completion times (host steady clock, seconds) are collected in `done`."""

    def __init__(self, agent, mem_budget=8 << 30, max_batch_obs=8192, n_slots=4):
        self.agent = agent
        self.done = {}
        self._keep = {}
        self._cb = L.DONE_CB(self._on_done)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        check(L.LIB.sq_server_create(agent.handle, int(mem_budget), int(max_batch_obs), int(n_slots),
                                     ctypes.byref(h)))
        self.handle = h

    def _on_done(self, rid, t, _user):
        self.done[int(rid)] = float(t)
        self._keep.pop(int(rid), None)

    def submit(self, frames, proprio, request_id, sample=False, out=None):
        n = frames.shape[0]
        cfg = self.agent.cfg
        _req(frames, torch.uint8, (n, cfg["H"], cfg["W"], cfg["C"]), "frames")
        _req(proprio, torch.float32, (n, cfg["proprio"]), "proprio")
        if out is None:
            out = torch.empty((n, cfg["action"]), dtype=torch.float32, device=frames.device)
        self._keep[int(request_id)] = (frames, proprio, out)
        check(L.LIB.sq_server_submit(self.handle, ptr(frames), ptr(proprio), n, int(bool(sample)), int(request_id),
                                     ptr(out), self._cb, None))
        return out

    def drain(self):
        check(L.LIB.sq_server_drain(self.handle))

    def hold(self, on=True):
        """Pause (True) or resume (False) admissions; requests keep queueing."""
        check(L.LIB.sq_server_hold(self.handle, int(bool(on))))

    def stats(self):
        """Launch counters and the device busy time of the completed batches."""
        st = L.ServerStats()
        check(L.LIB.sq_server_get_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in L.ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            L.LIB.sq_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
