/* squint.h -- C ABI of libsquint, an MI355X (gfx950) implementation of the
 * batched visual Soft Actor-Critic update of Squint (arXiv 2602.21203) and its
 * policy query.
 *
 * Conventions (apply to every call unless stated otherwise)
 *   Pointers      every T* is a DEVICE pointer unless marked [host].
 *   Ownership     the caller allocates and frees every buffer it passes; the
 *                 library only borrows them for the call (an sq_agent borrows
 *                 the buffers given to sq_agent_create for its lifetime).  The
 *                 library allocates device memory only in sq_agent_create,
 *                 sq_server_create, sq_ring_create, sq_env_create and when
 *                 sac_update captures a new graph, and frees it in the matching
 *                 *_destroy (or when the graph is evicted).
 *   Streams       calls are asynchronous on `stream` (a hipStream_t; NULL is the
 *                 null stream).  No call synchronises the device except the
 *                 sq_server_* host waits.
 *   Gradients     gradient outputs are overwritten, never accumulated.
 *   Errors        0 = SQ_OK.  SQ_EINVAL: bad argument, nothing was enqueued.
 *                 SQ_ENOMEM: allocation failed or a request exceeds a budget.
 *                 SQ_EDEVICE: a HIP runtime error (launch or API).
 *                 SQ_ECAPTURE: a call that cannot be captured was made while the
 *                 stream is capturing.  sq_last_error() returns a message for the
 *                 last failure on the calling thread.
 *   Precision     sq_prec selects how GEMM and convolution operands are rounded:
 *                 SQ_F32 multiplies FP32 operands; SQ_BF16 rounds weights,
 *                 activations and upstream gradients to bfloat16 (nearest even)
 *                 and accumulates in FP32.  LayerNorm, softmax, the categorical
 *                 projection, the tanh-Gaussian head and Adam are FP32 in both.
 *   Determinism   no kernel uses floating-point atomics; every reduction has a
 *                 fixed order, so a call is bitwise reproducible.
 *   Threads       an sq_agent must not be used by two threads at once.
 *
 * Layouts
 *   frames        [rows, H, W, C] uint8, HWC, channel c = 3*s + rgb for stack
 *                 slot s (oldest first).  H/k == W/k = S, the squinted side
 *                 (16, or 32 for the higher-resolution variant).
 *   images        [n, C, S, S] float (or bfloat16 bits), CHW.
 *   features      [n, flat] float, flattened (channel, y, x).
 *   parameters    one flat float vector in the canonical order reported by
 *                 sq_param_offsets (encoder convs, critic projection, twin
 *                 critic MLPs, actor projection, actor MLP, log alpha).  The
 *                 target critic is a copy of the critic block.
 */
#ifndef SQUINT_H
#define SQUINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define SQ_API __attribute__((visibility("default")))
#else
#define SQ_API
#endif

typedef struct ihipStream_t* sq_stream_t; /* identical to hipStream_t */

enum { SQ_OK = 0, SQ_EINVAL = 1, SQ_ENOMEM = 2, SQ_EDEVICE = 3, SQ_ECAPTURE = 4 };
typedef enum { SQ_F32 = 0, SQ_BF16 = 1 } sq_prec;

/* Network and data dimensions (Sec. IV: 16x16 network input reached by area
 * downsampling, a small conv encoder, LayerNorm MLPs, C51 critics).
 *   C        channels of a frame stack (3 per RGB frame)
 *   H, W, k  source frame size and squint factor; the network sees H/k x W/k
 *            (16 x 16 in the paper; 32 x 32 is its higher-resolution variant)
 *   n_conv   number of 3x3 valid convs (first has stride 2), 1..4
 *   F        conv channels; proj: projection width; hidden: MLP width
 *   atoms    C51 atoms on [v_min, v_max] (>= 2); atoms = 1 selects a scalar
 *            critic trained on the squared Bellman error (Eqs. (1)-(2)),
 *            v_min / v_max unused; proprio / action: vector sizes */
typedef struct {
  int C, H, W, k;
  int n_conv, F, proj, hidden, atoms, proprio, action;
  float v_min, v_max;
} sq_dims;

/* Update hyperparameters.  target_entropy is usually -action; log_std_min/max
 * bound the squashed log standard deviation of the policy; policy_freq delays
 * the actor step to updates u with u % policy_freq == 0 (u = global counter);
 * seed keys the Philox4x32-10 draws (replay indices, policy noise).  gamma must
 * lie in [0, 1] (sq_agent_create returns SQ_EINVAL otherwise). */
typedef struct {
  float gamma, lr, beta1, beta2, adam_eps, rho, target_entropy, log_std_min, log_std_max;
  int policy_freq;
  sq_prec prec;
  unsigned long long seed;
  int cdq;   /* 0: average the twin targets (the paper's choice); 1: clipped double-Q,
                the twin with the smaller expected value per row (Sec. IV Critic Design Choices) */
} sq_hparams;

/* Replay view, all device pointers, caller-owned; rows [0, size) are valid.
 * squinted = 0: frames are raw [capacity, H, W, C] and the update squints them.
 * squinted = 1: frames were squinted at insertion (sq_ring) and are stored as
 *   uint8 block means [capacity, H/k, W/k, C]; the update scales them by 1/255.
 * dev_size (nullable): device int holding the row count, read by every update
 *   in place of `size` (a ring that keeps growing between graph replays). */
typedef struct {
  const uint8_t* obs;          /* [capacity, H, W, C] or [capacity, H/k, W/k, C] */
  const uint8_t* next_obs;     /* same shape as obs */
  const float* proprio;        /* [capacity, proprio] */
  const float* next_proprio;   /* [capacity, proprio] */
  const float* action;         /* [capacity, action] */
  const float* reward;         /* [capacity] */
  const uint8_t* done;         /* [capacity], 0 or 1 */
  int capacity, size;
  int squinted;
  const int* dev_size;
} sq_replay;

typedef struct sq_agent sq_agent;
typedef struct sq_server sq_server;
typedef struct sq_ring sq_ring;

/* ---------------------------------------------------------------- host-side */
SQ_API const char* sq_last_error(void);
SQ_API int sq_version(void);

/* Number of floats in the flat parameter vector.  n: [host]. */
SQ_API int sq_param_count(const sq_dims* dims, long long* n);
/* Number of tensors in the canonical layout.  count: [host]. */
SQ_API int sq_param_tensor_count(const sq_dims* dims, int* count);
/* Offsets (in floats) of every tensor, canonical order, plus the end: off has
 * count + 1 entries [host].  Also reports the block boundaries [host, 4 each]:
 * blocks = {enc_begin, critic_begin, actor_begin, log_alpha}. */
SQ_API int sq_param_offsets(const sq_dims* dims, long long* off, long long* blocks);

enum { SQ_OP_ENCODER = 0, SQ_OP_CRITIC = 1, SQ_OP_ACTOR = 2 };
/* Bytes of workspace that encoder_*, critic_* or actor_* need for n rows. */
SQ_API int sq_workspace_bytes(const sq_dims* dims, int op, int n, size_t* bytes);

/* ---------------------------------------------------------------- operations */

/* Resolution squinting (Sec. IV Resolution Squinting; Alg. 1 downsampling):
 * mean of every disjoint k x k block, scaled to [-0.5, 0.5]:
 *   S = exact integer block sum, x = fl32(fl32(S / (255 k^2)) - 0.5).
 * frames: [rows, H, W, C] uint8; idx: [n] row indices into frames (NULL = rows
 * 0..n-1; every index must be in [0, rows), not checked on the device);
 * out: [n, C, S, S], float (out_prec SQ_F32) or bfloat16 bits (SQ_BF16,
 * rounded to nearest even from the FP32 value). */
SQ_API int squint_downsample(const sq_dims* dims, const uint8_t* frames, const int* idx, int n, sq_prec out_prec,
                      void* out, sq_stream_t stream);

/* Shared conv encoder f_psi (Sec. III; Sec. IV Encoder Design Choices): n_conv
 * 3x3 valid convolutions, the first with stride 2, each followed by ReLU.
 * enc_params: the encoder block of the flat vector; x: [n, C, S, S] float (also
 * under SQ_BF16: that form rounds x to bfloat16 once, as it stages it in LDS);
 * feat: [n, flat] float.  ws: sq_workspace_bytes(SQ_OP_ENCODER, n) bytes; it
 * keeps the activations for encoder_bwd and must not change in between. */
SQ_API int encoder_fwd(const sq_dims* dims, sq_prec prec, const float* enc_params, const float* x, int n,
                float* feat, void* ws, sq_stream_t stream);
/* encoder_fwd for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and the same feat bits, with the scratch
 * (rearranged weights, inner activations) in a fixed 16 MiB array that each
 * device holds from the library's first use until the process ends.  Keeps no
 * activations for encoder_bwd.  n above sq_encoder_noalloc_max_images returns
 * SQ_ENOMEM with nothing enqueued.  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams or threads) race and
 * must be ordered by the caller.  Allocates nothing. */
SQ_API int encoder_fwd_noalloc(const sq_dims* dims, sq_prec prec, const float* enc_params, const float* x, int n,
                               float* feat, sq_stream_t stream);
/* Largest n encoder_fwd_noalloc accepts for these dims.  n: [host]. */
SQ_API int sq_encoder_noalloc_max_images(const sq_dims* dims, int* n);
/* Gradient of the encoder parameters for upstream dfeat [n, flat] (same n as the
 * forward).  denc_params: encoder block of a flat gradient vector.  The image
 * receives no gradient. */
SQ_API int encoder_bwd(const sq_dims* dims, sq_prec prec, const float* enc_params, const void* ws, const float* dfeat,
                int n, float* denc_params, sq_stream_t stream);

/* Twin C51 critics (Sec. IV Critic Design Choices, Normalization; Alg. 1):
 * h = tanh(LN(W_c feat + b)); per twin i: ReLU(LN(L2(ReLU(LN(L1 [h; s; a])))))
 * -> atoms logits.  critic_params: the critic block (projection + both twins),
 * either online or target parameters.  feat [n, flat], proprio [n, P],
 * action [n, A]; logits [2, n, atoms].  ws: SQ_OP_CRITIC bytes. */
SQ_API int critic_fwd(const sq_dims* dims, sq_prec prec, const float* critic_params, const float* feat,
               const float* proprio, const float* action, int n, float* logits, void* ws, sq_stream_t stream);
/* Backward of critic_fwd for upstream dlogits [2, n, atoms].  Outputs (each
 * nullable): dparams (critic block layout), dfeat [n, flat], daction [n, A]. */
SQ_API int critic_bwd(const sq_dims* dims, sq_prec prec, const float* critic_params, const void* ws,
               const float* dlogits, int n, float* dparams, float* dfeat, float* daction, sq_stream_t stream);

/* Categorical (C51) projection of the soft Bellman target (Eq. (1) in
 * distributional form; Sec. IV Critic Design Choices):
 *   z_j = v_min + j dz, Tz_j = r + gamma (1 - d)(z_j + bonus),
 *   b_j = clamp((Tz_j - v_min) / dz, 0, N - 1),
 *   m_i = sum_j p_j max(0, 1 - |b_j - i|).
 * p_next [n, atoms], reward [n], done [n] uint8, bonus [n] (nullable = 0; the
 * update passes -alpha log pi(a'|s')), m [n, atoms].  FP32. */
SQ_API int c51_project(const sq_dims* dims, const float* p_next, const float* reward, const uint8_t* done,
                const float* bonus, float gamma, int n, float* m, sq_stream_t stream);

/* Tanh-Gaussian actor (Sec. III Eq. (3)): h = tanh(LN(W_a feat + b)); MLP on
 * [h; s] -> [mu, u_s]; log sigma = lo + (hi - lo)(tanh(u_s) + 1)/2;
 * u = mu + sigma eps; action = tanh(u);
 * log pi = sum_d (-eps_d^2/2 - log sigma_d - log(2 pi)/2 - log(1 - tanh(u_d)^2)).
 * actor_params: the actor block.  eps [n, A] standard normal (NULL: the mean
 * action tanh(mu), logp not written).  action [n, A]; logp [n] (nullable).
 * ws: SQ_OP_ACTOR bytes, kept for actor_bwd. */
SQ_API int actor_fwd(const sq_dims* dims, sq_prec prec, const sq_hparams* hp, const float* actor_params,
              const float* feat, const float* proprio, const float* eps, int n, float* action, float* logp,
              void* ws, sq_stream_t stream);
/* Backward of a sampled actor_fwd for upstream daction [n, A] and dlogp [n]
 * (nullable = 0).  dparams: actor block layout.  No gradient to feat. */
SQ_API int actor_bwd(const sq_dims* dims, sq_prec prec, const sq_hparams* hp, const float* actor_params,
              const void* ws, const float* daction, const float* dlogp, int n, float* dparams,
              sq_stream_t stream);

/* Adam with bias correction (the paper's gradient steps, read as Adam):
 *   t = *step + 1,
 *   m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * then *step = t (a one-thread launch ordered after the update on `stream`).
 * Optionally updates an EMA target (Alg. 1 target update) for i >= ema_begin:
 *   ema_target[i - ema_begin] = rho ema_target[i - ema_begin] + (1 - rho) p_new[i],
 * and writes bfloat16 bits of p_new to p_bf16.  n elements (n = 0 only advances
 * the counter); step: [1] int, device. */
SQ_API int adam_step(float* p, const float* g, float* m, float* v, long long n, const sq_hparams* hp,
              int* step, uint16_t* p_bf16, float* ema_target, long long ema_begin, sq_stream_t stream);

/* Batched dense product on the matrix cores, the building block of every
 * linear layer above (exposed for tests and measurement):
 *   C[z](r, c) (+)= sum_k A[z](r, k) * B[z](c, k) + bias[z][c]
 * with A[z](r, k) = A[z*a_sz + r*a_lr + k*a_lk] and B[z](c, k) likewise; C is
 * row-major with leading dimension ldc.  SQ_BF16 rounds A and B to bfloat16;
 * accumulation is FP32 in a fixed order.  bias nullable; accumulate adds to C. */
SQ_API int sq_gemm(sq_prec prec, int M, int N, int K, int batch, const float* A, long long a_lr, long long a_lk,
                   long long a_sz, const float* B, long long b_lr, long long b_lk, long long b_sz, float* C,
                   long long ldc, long long c_sz, const float* bias, long long bias_sz, int accumulate,
                   sq_stream_t stream);

/* ---------------------------------------------------------------- agent */

/* An agent bundles the caller's state buffers and the library's workspace for
 * batch `batch`:
 *   params [n], target [critic block size], adam_m, adam_v [n]: float;
 *   grads [n] float (nullable: internal), written by every update;
 *   counters [4] int: {u, critic+encoder Adam steps, actor steps, alpha steps}.
 * The caller initialises params, sets target = critic block of params, zeroes
 * the moments and counters. */
SQ_API int sq_agent_create(const sq_dims* dims, const sq_hparams* hp, int batch, float* params, float* target,
                    float* adam_m, float* adam_v, float* grads, int* counters, sq_agent** out /*[host]*/);
SQ_API int sq_agent_destroy(sq_agent* agent);
/* The agent keeps a packed copy of the linear weights (rows padded and aligned
 * for 16-byte loads) that its updates refresh.  After the caller changes params
 * or target itself (e.g. loading a checkpoint), call sq_agent_sync before the
 * next sac_update or act. */
SQ_API int sq_agent_sync(sq_agent* agent, sq_stream_t stream);

/* n_updates SAC updates (Alg. 1 inner loop, with the readings stated in the
 * design notes): per update, draw batch replay indices and noise from Philox
 * keyed by (seed, u), squint obs and next_obs, encode both, build the C51 soft
 * target from the averaged twin target critics, step critic + encoder on the
 * summed cross entropy, step log alpha, step the actor when u % policy_freq
 * == 0, update the target EMA, write stats[u_local, 0..7] = {critic loss,
 * actor loss, alpha loss, alpha, entropy, mean Q, mean target, non-finite}.
 * The first call for a given (n_updates, replay contents, stream, policy_freq
 * phase) captures a HIP graph and allocates its [n_updates, 8] statistics buffer;
 * later calls with the same key replay the graph and copy the statistics to
 * `stats` (so `stats` may differ between calls).  At most 8 graphs are kept per
 * agent: a miss beyond that destroys the least recently used one after a device
 * synchronisation.  A non-finite statistic (stats[u, 7] = 1, e.g. from a NaN
 * reward) does not stop the update: the parameters take the non-finite step as
 * computed, and the caller restores them.  stats: [n_updates, 8] float.
 * Inside a caller's capture the kernels are recorded into that graph directly. */
SQ_API int sac_update(sq_agent* agent, const sq_replay* replay, int n_updates, float* stats, sq_stream_t stream);
/* The same sequence launched kernel by kernel, without a graph. */
SQ_API int sac_update_eager(sq_agent* agent, const sq_replay* replay, int n_updates, float* stats, sq_stream_t stream);

/* Policy query (Alg. 1 action sampling): squint frames [n, H, W, C] uint8,
 * encode, actor mean (sample = 0) or tanh-Gaussian sample (sample = 1, noise
 * keyed by (seed, request_id, row)) -> action_out [n, A].  BF16 operands when
 * hp.prec is SQ_BF16.  n <= the agent's act capacity (see sq_agent_act_capacity). */
SQ_API int act(sq_agent* agent, const uint8_t* frames, const float* proprio, int n, int sample,
        unsigned long long request_id, float* action_out, sq_stream_t stream);
SQ_API int sq_agent_act_capacity(sq_agent* agent, int* n /*[host]*/);

/* ---------------------------------------------------------------- insert path */
/* GPU FIFO replay of squinted transitions (Alg. 1: each observation is
 * downsampled when observed and the downsampled pair is what the buffer stores;
 * Sec. V Replay Buffer Size: a simple FIFO held on the GPU).
 * sq_ring_create allocates capacity rows (device memory, zero-filled; about
 * 2 (H/k)(W/k) C + 4 (2 proprio + action + 1) + 1 bytes per row) and owns them
 * until sq_ring_destroy.  capacity in [1, 2^31 - 1]. */
SQ_API int sq_ring_create(const sq_dims* dims, int capacity, sq_ring** out);
SQ_API int sq_ring_destroy(sq_ring* ring);
/* Squint n transitions at insertion and append them: obs, next_obs [n, H, W, C]
 * uint8 raw frames; proprio, next_proprio [n, proprio], action [n, A], reward [n]
 * float; done [n] uint8 (all device pointers, read only).  Each frame is stored
 * as its k x k block means, q = nearest integer to S / k^2 with ties to even
 * (S the exact integer block sum), [H/k, W/k, C] uint8.  Transition i lands in
 * row (pos + i) % capacity; then pos = (pos + n) % capacity and size =
 * min(size + n, capacity).  n in [0, capacity] (SQ_EINVAL otherwise).  The write
 * position is kept on the host, so the call cannot be captured (SQ_ECAPTURE);
 * the row count the update samples from is also kept on the device. */
SQ_API int sq_ring_insert(sq_ring* ring, const uint8_t* obs, const uint8_t* next_obs, const float* proprio,
                          const float* next_proprio, const float* action, const float* reward, const uint8_t* done,
                          int n, sq_stream_t stream);
/* A replay view of the ring for sac_update: squinted = 1, dev_size set (and
 * size = capacity, unused), so one captured graph keeps sampling the whole ring
 * as it grows.  Sampling an empty ring reads its zero-filled rows.  out: [host]. */
SQ_API int sq_ring_view(const sq_ring* ring, sq_replay* out);
/* Host copy of the write position and row count after the inserts enqueued so
 * far.  pos, size: [host]. */
SQ_API int sq_ring_state(const sq_ring* ring, int* pos, int* size);
/* Copy rows [row0, row0 + n) of one stored field into dst (device or host
 * memory, caller-owned, densely packed rows), ordered on `stream`
 * (hipMemcpyAsync; host dst needs a stream synchronisation before use).
 * field: SQ_RING_OBS, SQ_RING_NEXT_OBS (uint8 [side, side, C] rows),
 * SQ_RING_PROPRIO, SQ_RING_NEXT_PROPRIO, SQ_RING_ACTION, SQ_RING_REWARD (float
 * rows), SQ_RING_DONE (uint8).  SQ_EINVAL when the rows leave [0, capacity). */
enum { SQ_RING_OBS = 0, SQ_RING_NEXT_OBS = 1, SQ_RING_PROPRIO = 2, SQ_RING_NEXT_PROPRIO = 3, SQ_RING_ACTION = 4,
       SQ_RING_REWARD = 5, SQ_RING_DONE = 6 };
SQ_API int sq_ring_copy_out(const sq_ring* ring, int field, int row0, int n, void* dst, sq_stream_t stream);

/* ---------------------------------------------------------------- environment stub */
/* A synthetic stand-in for the simulator of Alg. 1's outer loop (observe, act,
 * step, store, then the UTD updates), so that the loop runs end to end on the
 * device: per environment a point mass s[P] (P = proprio, 2..12) driven by the
 * action (s_j <- clamp(s_j + a_{j mod A} / 8, -2, 2)), reward -|s_{0,1} - goal|^2,
 * episodes of episode_len steps with Philox-drawn resets, and an integer
 * renderer that draws the last three positions as discs into the frame stack
 * ([n, H, W, C] uint8, C = 3, 6 or 9, H and W powers of two >= 8).
 * sq_env_create allocates the state and buffers and resets every environment. */
typedef struct sq_env sq_env;
/* Caller-owned device buffers of the environments (n = n_envs, P = proprio). */
typedef struct {
  uint8_t* obs[2];        /* [n, H, W, C] observation buffers, used in turn: obs[k] is
                             current after an even (k = 0) or odd (k = 1) number of steps */
  float* proprio;         /* [n, P] current proprio (the environment state) */
  uint8_t* next_obs;      /* [n, H, W, C] last transition's next observation */
  float* proprio_t;       /* [n, P] last transition's proprio */
  float* next_proprio;    /* [n, P] last transition's next proprio */
  float* reward;          /* [n] */
  uint8_t* done;          /* [n] */
} sq_env_buffers;
/* Allocates the small per-environment state (goal, step, episode, frame stack),
 * resets every environment into obs[0] / proprio, and keeps the buffer pointers
 * (the caller keeps the memory alive until sq_env_destroy). */
SQ_API int sq_env_create(const sq_dims* dims, int n_envs, int episode_len, unsigned long long seed,
                         const sq_env_buffers* bufs, sq_env** out);
SQ_API int sq_env_destroy(sq_env* env);
/* One step of every environment with action [n, A] (device): writes the
 * transition (the previous current observation stays in its buffer as the
 * transition's observation; next_obs, proprio_t, next_proprio, reward, done) and
 * the next observation into the other obs buffer, which becomes current.  Store
 * the transition before the next step, which overwrites that buffer.  The
 * buffer parity is kept on the host, so the call cannot be captured (SQ_ECAPTURE). */
SQ_API int sq_env_step(sq_env* env, const float* action, sq_stream_t stream);

/* ---------------------------------------------------------------- serving */
typedef void (*sq_done_cb)(unsigned long long request_id, double t_done_s, void* user);
/* Continuous-batching act() server (Alg. 1 action sampling for many environment
 * pools): a host scheduler thread fuses queued requests (FIFO, no skipping) into
 * one launch on a free stream slot when the batch's rows stay within
 * max_batch_obs and its workspace fits the memory budget still free; batches
 * on different slots overlap on the device.  A host function enqueued after each
 * batch wakes the scheduler (no polling).  Each row's result does not depend on
 * the rows it shares a launch with, so a request gets the same bits alone or in
 * any mix.  The server reads the agent's weights in place (no copy). */
SQ_API int sq_server_create(sq_agent* agent, size_t mem_budget, int max_batch_obs, int n_slots, sq_server** out);
/* Queue one request of n observations (frames [n, H, W, C] uint8, proprio [n, P],
 * device; action_out [n, A], device).  The buffers must stay valid until the
 * callback (host steady-clock completion time in seconds) has run. */
SQ_API int sq_server_submit(sq_server* srv, const uint8_t* frames, const float* proprio, int n, int sample,
                     unsigned long long request_id, float* action_out, sq_done_cb cb, void* user);
/* Block until every queued request has completed and its callback returned. */
SQ_API int sq_server_drain(sq_server* srv);
/* hold = 1 pauses admissions (requests keep queueing), hold = 0 resumes them. */
SQ_API int sq_server_hold(sq_server* srv, int hold);
typedef struct {
  long long batches;               /* launches */
  long long requests, rows;        /* requests and observations launched */
  long long fused_batches;         /* launches that fused two or more requests */
  int max_requests_per_batch;
  int max_slots_busy;              /* most slots holding a batch at once */
  long long overlapped_batches;    /* batches whose device interval began before an earlier one ended */
  double device_busy_s;            /* union of the batches' device intervals (timing events) */
  double device_span_s;            /* first batch start to last batch end on the device */
} sq_server_stats;
/* Counters since sq_server_create (completed batches for the device times). */
SQ_API int sq_server_get_stats(sq_server* srv, sq_server_stats* out /*[host]*/);
SQ_API int sq_server_destroy(sq_server* srv);

/* ---------------------------------------------------------------- test hooks */
/* Graphs captured by sac_update so far, and graphs currently cached.  [host] */
SQ_API int sq_agent_graph_count(const sq_agent* agent, long long* captured, int* cached);
/* Copy of the replay rows drawn by the agent's last enqueued update (idx [batch]
 * int, device), ordered on `stream` after that update. */
SQ_API int sq_agent_last_indices(const sq_agent* agent, int* idx, sq_stream_t stream);
/* Copy of the projected target distribution m of the agent's last enqueued
 * update (Eq. (1) in categorical form, the C51 projection of the twin-target
 * softmax: m [batch][atoms] float, device), ordered on `stream` after that update.
 * SQ_EINVAL for scalar critics (atoms = 1), which have no distribution. */
SQ_API int sq_agent_last_target(const sq_agent* agent, float* m, sq_stream_t stream);
/* Row of transition i of an insertion at write position pos in a ring of
 * `capacity` rows: (pos + i) mod capacity, in 64-bit arithmetic.  [host] */
SQ_API int sq_ring_row(int pos, long long i, int capacity, int* row);
/* Output tile (bx, by, bz) -> tile[0..2] that workgroup b of a gx x gy x gz
 * linear-layer product grid computes (the XCD-aware order the product kernels
 * use).  [host] */
SQ_API int sq_gemm_tile_order(int b, int gx, int gy, int gz, int* tile);
/* bfloat16 operand copies.  With on = 1 (the default), an agent created in the
 * bfloat16 mode keeps bfloat16 copies of its packed weights and of the
 * activations its forward products read, written by their producers, and those
 * products read the copies: the same results, half the operand bytes.  With 0,
 * agents created afterwards keep none and their products round the FP32
 * operands.  Returns the previous setting.  [host] */
SQ_API int sq_bf16_operand_copies(int on);
/* Linear-layer products enqueued on bfloat16 copies so far in this process
 * (launches recorded into a graph count once, at capture).  [host] */
SQ_API int sq_bf16_copy_products(long long* n);
/* C[z](r, c) = sum_k A[z](r, k) B[z](c, k) (+ bias[z*bias_sz + c]) on bfloat16
 * operands (bit patterns), A[z](r, k) = A[z*a_sz + r*a_lr + k*a_lk] and B
 * likewise.  Each operand is either k-contiguous (lk = 1: rows 16-byte aligned,
 * holding K rounded up to 8 elements) or transposed (lr = 1: k-slices 16-byte
 * aligned, holding its row count rounded up to 8 elements).  The kernel of the
 * products that read bfloat16 copies; FP32 accumulation in the order of
 * sq_gemm's bfloat16 mode, so C equals sq_gemm's result on the FP32 values of A
 * and B. */
SQ_API int sq_gemm_bf16(int M, int N, int K, int batch, const uint16_t* A, long long a_lr, long long a_lk,
                        long long a_sz, const uint16_t* B, long long b_lr, long long b_lk, long long b_sz, float* C,
                        long long ldc, long long c_sz, const float* bias, long long bias_sz, sq_stream_t stream);
/* idx[b] = mulhi32(Philox4x32_10(ctr = (update, 0, b, 0), key = seed).w0, size). */
SQ_API int sq_sample_indices(unsigned long long seed, unsigned int update, int size, int n, int* idx,
                      sq_stream_t stream);
/* Box-Muller on Philox words (w0, w1) of ctr = (update, stream_id, e, 0):
 * eps[e] = sqrt(-2 ln u1) cos(2 pi u2), u = ((w >> 9) + 0.5) 2^-23 (exact in FP32). */
SQ_API int sq_gaussian(unsigned long long seed, unsigned int update, unsigned int stream_id, int n, float* eps,
                sq_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SQUINT_H */
