// Lifecycle of the synthetic environment stub (kernels/env.hip): the small
// per-environment state is library-owned; observation and transition buffers
// belong to the caller, and the two observation buffers are used in turn.
#include "ops.h"

using namespace sq;

struct sq_env {
  Net net;
  EnvState E;
  sq_env_buffers b;
  void* mem = nullptr;
  int cur = 0;
};

extern "C" {

int sq_env_create(const sq_dims* dims, int n_envs, int episode_len, unsigned long long seed,
                  const sq_env_buffers* bufs, sq_env** out) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  if (net.d.n_conv == 0) {
    set_error("state-based dims (n_conv = 0) have no frames to store");
    return SQ_EINVAL;
  }
  if (!out || !bufs || n_envs <= 0 || episode_len <= 0) {
    set_error("bad environment arguments (n_envs %d, episode_len %d)", n_envs, episode_len);
    return SQ_EINVAL;
  }
  if (!bufs->obs[0] || !bufs->obs[1] || !bufs->proprio || !bufs->next_obs || !bufs->proprio_t ||
      !bufs->next_proprio || !bufs->reward || !bufs->done) {
    set_error("NULL environment buffer");
    return SQ_EINVAL;
  }
  const sq_dims& d = net.d;
  const bool pow2 = (d.H & (d.H - 1)) == 0 && (d.W & (d.W - 1)) == 0;
  // the frame stack holds three positions: C <= 9 keeps every channel's slot in range
  if (d.proprio < 2 || d.proprio > 12 || d.C % 3 != 0 || d.C > 9 || !pow2 || d.H < 8 || d.W < 8) {
    set_error("the environment stub needs 2..12 proprio values, 3, 6 or 9 channels and power-of-two sides >= 8");
    return SQ_EINVAL;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
    set_error("sq_env_create allocates and cannot run while the null stream captures");
    return SQ_ECAPTURE;
  }
  sq_env* v = new sq_env;
  v->net = net;
  v->b = *bufs;
  const size_t n = (size_t)n_envs;
  Bump m{nullptr};
  m.take<float>(n * 2);
  m.take<int>(n);
  m.take<int>(n);
  m.take<int>(n * 6);
  if (hipMalloc(&v->mem, m.off + 256) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of the environment state failed");
    delete v;
    return SQ_ENOMEM;
  }
  Bump b{(char*)v->mem};
  float* g = b.take<float>(n * 2);
  int* t = b.take<int>(n);
  int* ep = b.take<int>(n);
  int* stack = b.take<int>(n * 6);
  v->E = EnvState{n_envs, d.H, d.W, d.C, d.proprio, d.action, episode_len, (unsigned)seed, (unsigned)(seed >> 32),
                  bufs->proprio, g, t, ep, stack};
  const int s = env_reset_all(v->E, bufs->obs[0], nullptr);
  if (s != SQ_OK || hipDeviceSynchronize() != hipSuccess) {
    set_error("environment reset failed");
    (void)hipFree(v->mem);
    delete v;
    return SQ_EDEVICE;
  }
  *out = v;
  return SQ_OK;
}

int sq_env_destroy(sq_env* v) {
  if (!v) return SQ_OK;
  if (v->mem) (void)hipFree(v->mem);
  delete v;
  return SQ_OK;
}

int sq_env_step(sq_env* v, const float* action, sq_stream_t stream) {
  if (!v || !action) { set_error("NULL argument to sq_env_step"); return SQ_EINVAL; }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    set_error("sq_env_step alternates its observation buffers on the host and cannot be captured");
    return SQ_ECAPTURE;
  }
  const sq_env_buffers& b = v->b;
  SQ_TRY(env_step(v->E, action, b.proprio_t, b.next_obs, b.next_proprio, b.reward, b.done, b.obs[v->cur ^ 1],
                  (hipStream_t)stream));
  v->cur ^= 1;
  return SQ_OK;
}

}  // extern "C"
