// C ABI entry points: argument validation, workspace carving, dispatch to the
// kernels.  On SQ_EINVAL nothing has been enqueued.
#include <string.h>

#include "ops.h"

namespace sq {
const char* last_error();
}

using namespace sq;

#define SQ_REQUIRE(cond, ...)          \
  do {                                 \
    if (!(cond)) {                     \
      ::sq::set_error(__VA_ARGS__);    \
      return SQ_EINVAL;                \
    }                                  \
  } while (0)

static bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

extern "C" {

const char* sq_last_error(void) { return last_error(); }

int sq_version(void) { return 1; }

int sq_param_count(const sq_dims* dims, long long* n) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(n, "n is NULL");
  Layout L;
  make_layout(net, &L);
  *n = L.total;
  return SQ_OK;
}

int sq_param_tensor_count(const sq_dims* dims, int* count) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(count, "count is NULL");
  Layout L;
  make_layout(net, &L);
  *count = L.n_tensors;
  return SQ_OK;
}

int sq_param_offsets(const sq_dims* dims, long long* off, long long* blocks) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  Layout L;
  make_layout(net, &L);
  if (off)
    for (int i = 0; i <= L.n_tensors; ++i) off[i] = L.tensor_off[i];
  if (blocks) {
    blocks[0] = L.enc_begin;
    blocks[1] = L.critic_begin;
    blocks[2] = L.actor_begin;
    blocks[3] = L.log_alpha;
  }
  return SQ_OK;
}

// standalone-op workspaces (saved activations persist from *_fwd to *_bwd)
struct EncWs { float* x; EncBufs e; };
struct CriticWs { float* feat; CriticBufs c; };
struct ActorWs { float* feat; float* eps; ActorBufs a; };

static size_t plan_op(const Net& net, int op, int n, char* base, void* out) {
  Bump b{base};
  if (op == SQ_OP_ENCODER) {
    EncWs w;
    w.x = b.take<float>((size_t)n * net.img);
    plan_encoder(net, n, b, &w.e, true);
    if (out) *(EncWs*)out = w;
  } else if (op == SQ_OP_CRITIC) {
    CriticWs w;
    w.feat = b.take<float>((size_t)n * net.flat);
    plan_critic(net, n, b, &w.c, true);
    if (out) *(CriticWs*)out = w;
  } else {
    ActorWs w;
    w.feat = b.take<float>((size_t)n * net.flat);
    w.eps = b.take<float>((size_t)n * net.d.action);
    plan_actor(net, n, b, &w.a, true);
    if (out) *(ActorWs*)out = w;
  }
  return b.off + 256;
}

int sq_workspace_bytes(const sq_dims* dims, int op, int n, size_t* bytes) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(op >= SQ_OP_ENCODER && op <= SQ_OP_ACTOR, "unknown op %d", op);
  SQ_REQUIRE(n >= 0 && bytes, "bad n or bytes");
  *bytes = plan_op(net, op, n, nullptr, nullptr);
  return SQ_OK;
}

static char* ws_base(void* ws) { return (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255) ; }

int squint_downsample(const sq_dims* dims, const uint8_t* frames, const int* idx, int n, sq_prec out_prec,
                      void* out, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(dims->n_conv > 0, "state-based dims (n_conv = 0) have no frames or encoder");
  SQ_REQUIRE(n >= 0, "n < 0");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(frames && out, "NULL frames or out");
  SQ_REQUIRE(out_prec == SQ_F32 ? aligned4(out) : (((uintptr_t)out & 1u) == 0), "misaligned out");
  return launch_squint(frames, idx, n, dims->H, dims->W, dims->C, dims->k, out_prec == SQ_BF16, out,
                       (long long)net.img, (hipStream_t)stream);
}

int encoder_fwd(const sq_dims* dims, sq_prec prec, const float* enc_params, const float* x, int n, float* feat,
                void* ws, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(dims->n_conv > 0, "state-based dims (n_conv = 0) have no frames or encoder");
  SQ_REQUIRE(n >= 0, "n < 0");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(enc_params && x && feat && ws, "NULL argument");
  SQ_REQUIRE(aligned4(enc_params) && aligned4(x) && aligned4(feat), "misaligned argument");
  Layout L;
  make_layout(net, &L);
  EncWs w;
  plan_op(net, SQ_OP_ENCODER, n, ws_base(ws), &w);
  hipStream_t st = (hipStream_t)stream;
  SQ_TRY_HIP(hipMemcpyAsync(w.x, x, (size_t)n * net.img * 4, hipMemcpyDeviceToDevice, st));
  SQ_TRY(encoder_forward(net, prec == SQ_BF16, enc_params, L, w.x, n, w.e, st));
  SQ_TRY_HIP(hipMemcpyAsync(feat, w.e.h[dims->n_conv - 1], (size_t)n * net.flat * 4, hipMemcpyDeviceToDevice, st));
  return SQ_OK;
}

int encoder_bwd(const sq_dims* dims, sq_prec prec, const float* enc_params, const void* ws, const float* dfeat, int n,
                float* denc_params, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(dims->n_conv > 0, "state-based dims (n_conv = 0) have no frames or encoder");
  SQ_REQUIRE(n >= 0, "n < 0");
  SQ_REQUIRE(enc_params && ws && denc_params && (dfeat || n == 0), "NULL argument");
  Layout L;
  make_layout(net, &L);
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) {
    SQ_TRY_HIP(hipMemsetAsync(denc_params, 0, (size_t)L.enc_end * 4, st));
    return SQ_OK;
  }
  EncWs w;
  plan_op(net, SQ_OP_ENCODER, n, ws_base((void*)ws), &w);
  return encoder_backward(net, prec == SQ_BF16, enc_params, L, w.x, n, dfeat, w.e, denc_params, st);
}

int critic_fwd(const sq_dims* dims, sq_prec prec, const float* critic_params, const float* feat, const float* proprio,
               const float* action, int n, float* logits, void* ws, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(n >= 0, "n < 0");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(critic_params && feat && action && logits && ws && (proprio || dims->proprio == 0), "NULL argument");
  Layout L;
  make_layout(net, &L);
  CriticWs w;
  plan_op(net, SQ_OP_CRITIC, n, ws_base(ws), &w);
  hipStream_t st = (hipStream_t)stream;
  SQ_TRY_HIP(hipMemcpyAsync(w.feat, feat, (size_t)n * net.flat * 4, hipMemcpyDeviceToDevice, st));
  return critic_forward(net, prec == SQ_BF16, critic_params, nullptr, L, w.feat, net.flat, proprio, dims->proprio, action,
                        dims->action, n, logits, w.c, st);
}

int critic_bwd(const sq_dims* dims, sq_prec prec, const float* critic_params, const void* ws, const float* dlogits,
               int n, float* dparams, float* dfeat, float* daction, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(n > 0, "n must be positive");
  SQ_REQUIRE(critic_params && ws && dlogits, "NULL argument");
  Layout L;
  make_layout(net, &L);
  CriticWs w;
  plan_op(net, SQ_OP_CRITIC, n, ws_base((void*)ws), &w);
  return critic_backward(net, prec == SQ_BF16, critic_params, nullptr, L, w.feat, net.flat, dlogits, n, w.c, dparams, dfeat,
                         daction, (hipStream_t)stream);
}

int c51_project(const sq_dims* dims, const float* p_next, const float* reward, const uint8_t* done, const float* bonus,
                float gamma, int n, float* m, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(n >= 0, "n < 0");
  SQ_REQUIRE(dims->atoms >= 2, "c51_project needs a categorical critic (atoms >= 2)");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(p_next && reward && done && m, "NULL argument");
  return c51_project_raw(p_next, reward, done, bonus, gamma, n, dims->atoms, dims->v_min, dims->v_max, m,
                         (hipStream_t)stream);
}

int actor_fwd(const sq_dims* dims, sq_prec prec, const sq_hparams* hp, const float* actor_params, const float* feat,
              const float* proprio, const float* eps, int n, float* action, float* logp, void* ws,
              sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(hp, "hp is NULL");
  SQ_REQUIRE(n >= 0, "n < 0");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(actor_params && feat && action && ws && (proprio || dims->proprio == 0), "NULL argument");
  Layout L;
  make_layout(net, &L);
  ActorWs w;
  plan_op(net, SQ_OP_ACTOR, n, ws_base(ws), &w);
  hipStream_t st = (hipStream_t)stream;
  SQ_TRY_HIP(hipMemcpyAsync(w.feat, feat, (size_t)n * net.flat * 4, hipMemcpyDeviceToDevice, st));
  if (eps) SQ_TRY_HIP(hipMemcpyAsync(w.eps, eps, (size_t)n * dims->action * 4, hipMemcpyDeviceToDevice, st));
  return actor_forward(net, prec == SQ_BF16, actor_params, nullptr, L, w.feat, net.flat, proprio, dims->proprio,
                       eps ? w.eps : nullptr, n, hp->log_std_min, hp->log_std_max, action, logp, w.a, st);
}

int actor_bwd(const sq_dims* dims, sq_prec prec, const sq_hparams* hp, const float* actor_params, const void* ws,
              const float* daction, const float* dlogp, int n, float* dparams, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  SQ_REQUIRE(hp, "hp is NULL");
  SQ_REQUIRE(n > 0, "n must be positive");
  SQ_REQUIRE(actor_params && ws && dparams, "NULL argument");
  Layout L;
  make_layout(net, &L);
  ActorWs w;
  plan_op(net, SQ_OP_ACTOR, n, ws_base((void*)ws), &w);
  return actor_backward(net, prec == SQ_BF16, actor_params, nullptr, L, w.feat, net.flat, w.eps, n, daction, dims->action,
                        dlogp, nullptr, 0.f, hp->log_std_min, hp->log_std_max, w.a, dparams, (hipStream_t)stream);
}

int adam_step(float* p, const float* g, float* m, float* v, long long n, const sq_hparams* hp, int* step,
              uint16_t* p_bf16, float* ema_target, long long ema_begin, sq_stream_t stream) {
  SQ_REQUIRE(hp, "hp is NULL");
  SQ_REQUIRE(n >= 0, "n < 0");
  SQ_REQUIRE(step, "step is NULL");
  if (n > 0) {
    SQ_REQUIRE(p && g && m && v, "NULL argument");
    SQ_REQUIRE(ema_begin >= 0 && ema_begin <= n, "ema_begin out of range");
    SQ_TRY(adam(p, g, m, v, n, hp, step, ema_target, ema_begin, p_bf16, nullptr, (hipStream_t)stream));
  }
  return launch_step_advance(step, (hipStream_t)stream);
}

int sq_gemm(sq_prec prec, int M, int N, int K, int batch, const float* A, long long a_lr, long long a_lk,
            long long a_sz, const float* B, long long b_lr, long long b_lk, long long b_sz, float* C, long long ldc,
            long long c_sz, const float* bias, long long bias_sz, int accumulate, sq_stream_t stream) {
  SQ_REQUIRE(M >= 0 && N >= 0 && K >= 0 && batch >= 0, "negative size");
  if (M == 0 || N == 0 || batch == 0) return SQ_OK;
  SQ_REQUIRE(C && (K == 0 || (A && B)), "NULL argument");
  SQ_REQUIRE(ldc >= N, "ldc < N");
  MatArg a{A, a_lr, a_lk, a_sz};
  MatArg b{B, b_lr, b_lk, b_sz};
  OutArg c{C, ldc, c_sz, bias, bias_sz, accumulate, 0};
  return gemm(prec == SQ_BF16, M, N, K, batch, a, b, c, nullptr, 0, (hipStream_t)stream);
}

int sq_bf16_operand_copies(int on) { return set_twins_enabled(on); }

int sq_bf16_copy_products(long long* n) {
  SQ_REQUIRE(n, "n is NULL");
  *n = copy_products();
  return SQ_OK;
}

int sq_gemm_bf16(int M, int N, int K, int batch, const uint16_t* A, long long a_lr, long long a_lk, long long a_sz,
                 const uint16_t* B, long long b_lr, long long b_lk, long long b_sz, float* C, long long ldc,
                 long long c_sz, const float* bias, long long bias_sz, sq_stream_t stream) {
  SQ_REQUIRE(M >= 0 && N >= 0 && K >= 0 && batch >= 0, "negative size");
  if (M == 0 || N == 0 || batch == 0) return SQ_OK;
  SQ_REQUIRE(K > 0, "sq_gemm_bf16 needs K > 0");
  SQ_REQUIRE(C && ldc >= N, "NULL C or ldc < N");
  OutArg c{C, ldc, c_sz, bias, bias_sz, 0, 0};
  return gemm_bf16_stored(M, N, K, batch, A, a_lr, a_lk, a_sz, B, b_lr, b_lk, b_sz, c, (hipStream_t)stream);
}

int sq_gemm_tile_order(int b, int gx, int gy, int gz, int* tile) {
  if (!tile || gx <= 0 || gy <= 0 || gz <= 0 || b < 0 || (long long)gx * gy * gz > (1LL << 30) ||
      b >= gx * gy * gz) {
    set_error("sq_gemm_tile_order: need a grid of positive sizes, 0 <= b < gx gy gz and a tile pointer");
    return SQ_EINVAL;
  }
  tile_of(b, gx, gy, gz, tile[0], tile[1], tile[2]);
  return SQ_OK;
}

int sq_sample_indices(unsigned long long seed, unsigned int update, int size, int n, int* idx, sq_stream_t stream) {
  SQ_REQUIRE(size > 0 && n >= 0, "need size > 0 and n >= 0");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(idx, "idx is NULL");
  return launch_indices(seed, update, size, n, idx, (hipStream_t)stream);
}

int sq_gaussian(unsigned long long seed, unsigned int update, unsigned int stream_id, int n, float* eps,
                sq_stream_t stream) {
  SQ_REQUIRE(n >= 0, "n < 0");
  if (n == 0) return SQ_OK;
  SQ_REQUIRE(eps, "eps is NULL");
  return launch_gaussian(seed, update, stream_id, n, eps, (hipStream_t)stream);
}

}  // extern "C"
