// Continuous-batching act() server.
//
// Requests (a pool of observations each, any size up to max_batch_obs) are
// queued FIFO.  A scheduler thread fuses every queued request that fits into
// one launch on a free stream slot: it fits while the fused row count stays
// within max_batch_obs and the in-flight activation memory (rows x bytes per
// observation) stays within the memory budget.  The head of the queue is never
// skipped.  Batches on different slots overlap on the device.  Rows reach their
// request's buffers through per-row pointer tables, and each row's result does
// not depend on which rows share its launch (no split reductions in the
// forward pass, noise keyed by (request id, row)), so a request gets the same
// bits alone or in any mix.
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "ops.h"

namespace sq {
const Net& agent_net(const sq_agent* g);
const Layout& agent_layout(const sq_agent* g);
const sq_hparams& agent_hp(const sq_agent* g);
const float* agent_params(const sq_agent* g);
const float* agent_pack(const sq_agent* g);
}  // namespace sq

using namespace sq;

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

namespace {

struct Req {
  const uint8_t* frames; const float* proprio; int n; int sample;
  unsigned long long id; float* out; sq_done_cb cb; void* user;
};

// per-row tables, one contiguous block (host pinned mirror + device copy)
struct Tables {
  const uint8_t** frames; const float** prop; float** out; unsigned long long* ids; int* rows; int* sample;
};
size_t tables_bytes(int cap) { return (size_t)cap * (8 + 8 + 8 + 8 + 4 + 4) + 64; }
Tables carve_tables(char* base, int cap) {
  Tables t;
  t.frames = (const uint8_t**)base;
  t.prop = (const float**)(base + (size_t)cap * 8);
  t.out = (float**)(base + (size_t)cap * 16);
  t.ids = (unsigned long long*)(base + (size_t)cap * 24);
  t.rows = (int*)(base + (size_t)cap * 32);
  t.sample = (int*)(base + (size_t)cap * 36);
  return t;
}

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  void* dmem = nullptr;
  char* htab = nullptr;
  char* dtab = nullptr;
  ActBufs w;
  float* prop_stage = nullptr;
  float* act_stage = nullptr;
  std::vector<Req> batch;
  bool busy = false;
  size_t bytes = 0;
};

}  // namespace

struct sq_server {
  sq_agent* agent;
  Net net;
  Layout L;
  sq_hparams hp;
  const float* params;
  size_t budget, per_obs, in_flight = 0;
  int max_batch;
  std::vector<Slot> slots;
  std::deque<Req> queue;
  std::mutex mu;
  std::condition_variable cv, idle;
  std::thread th;
  bool stop = false;
  size_t firing = 0;   // completions whose callbacks are running
  int error = SQ_OK;
  char errmsg[256] = {0};
};

static int launch_batch(sq_server* s, Slot& sl) {
  const sq_dims& d = s->net.d;
  const int cap = s->max_batch;
  Tables h = carve_tables(sl.htab, cap);
  const long long frame_bytes = (long long)d.H * d.W * d.C;
  int r = 0;
  for (const Req& q : sl.batch)
    for (int i = 0; i < q.n; ++i, ++r) {
      h.frames[r] = q.frames ? q.frames + (long long)i * frame_bytes : nullptr;
      h.prop[r] = q.proprio ? q.proprio + (long long)i * d.proprio : nullptr;
      h.out[r] = q.out + (long long)i * d.action;
      h.ids[r] = q.id;
      h.rows[r] = i;
      h.sample[r] = q.sample;
    }
  const int n = r;
  Tables t = carve_tables(sl.dtab, cap);
  hipStream_t st = sl.st;
  SQ_TRY_HIP(hipMemcpyAsync(sl.dtab, sl.htab, tables_bytes(cap), hipMemcpyHostToDevice, st));
  const int bf = s->hp.prec == SQ_BF16;
  if (d.n_conv > 0) {
    SQ_TRY(launch_squint_rows(t.frames, n, d.H, d.W, d.C, d.k, sl.w.x, st));
    SQ_TRY(encoder_forward(s->net, bf, s->params, s->L, sl.w.x, n, sl.w.e, st));
  }
  if (d.proprio > 0) SQ_TRY(gather_rows((const float* const*)t.prop, d.proprio, n, sl.prop_stage, st));
  SQ_TRY(act_noise_rows(s->hp.seed, t.ids, t.rows, t.sample, n, d.action, sl.w.noise, st));
  // state-based: the gathered states are the features
  const float* feat = d.n_conv > 0 ? sl.w.e.h[d.n_conv - 1] : sl.prop_stage;
  SQ_TRY(actor_forward(s->net, bf, s->params + s->L.actor_begin, agent_pack(s->agent), s->L, feat,
                       s->net.flat,
                       sl.prop_stage, d.proprio, sl.w.noise, n, s->hp.log_std_min, s->hp.log_std_max, sl.act_stage,
                       nullptr, sl.w.a, st));
  SQ_TRY(scatter_rows(sl.act_stage, d.action, n, t.out, st));
  SQ_TRY_HIP(hipEventRecord(sl.ev, st));
  return SQ_OK;
}

static void scheduler(sq_server* s) {
  std::vector<Req> done;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // completions
    bool any_busy = false;
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipSuccess) {
        for (const Req& r : sl.batch) done.push_back(r);
        sl.batch.clear();
        sl.busy = false;
        s->in_flight -= sl.bytes;
        sl.bytes = 0;
      } else if (q != hipErrorNotReady) {
        s->error = SQ_EDEVICE;
        snprintf(s->errmsg, sizeof(s->errmsg), "act batch failed: %s", hipGetErrorString(q));
        sl.busy = false;
        s->in_flight -= sl.bytes;
        sl.bytes = 0;
        sl.batch.clear();
      } else {
        any_busy = true;
      }
    }
    // admissions: FIFO, fuse every head request that fits
    for (Slot& sl : s->slots) {
      if (sl.busy || s->queue.empty()) continue;
      int rows = 0;
      while (!s->queue.empty()) {
        const Req& q = s->queue.front();
        const size_t need = (size_t)(rows + q.n) * s->per_obs;
        if (rows + q.n > s->max_batch || s->in_flight + need > s->budget) break;
        rows += q.n;
        sl.batch.push_back(q);
        s->queue.pop_front();
      }
      if (rows == 0) break;   // the head does not fit yet: wait for completions
      sl.bytes = (size_t)rows * s->per_obs;
      s->in_flight += sl.bytes;
      sl.busy = true;
      any_busy = true;
      if (launch_batch(s, sl) != SQ_OK) {
        s->error = SQ_EDEVICE;
        snprintf(s->errmsg, sizeof(s->errmsg), "%s", sq_last_error());
      }
    }
    if (!done.empty()) {
      std::vector<Req> fire;
      fire.swap(done);
      s->firing = fire.size();
      lk.unlock();
      const double t = now_s();
      for (const Req& r : fire)
        if (r.cb) r.cb(r.id, t, r.user);
      lk.lock();
      s->firing = 0;
      continue;
    }
    if (!any_busy && s->queue.empty()) {
      s->idle.notify_all();
      if (s->stop) break;
      s->cv.wait(lk);
      continue;
    }
    // a batch is on the device: poll its completion shortly
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::microseconds(20));
    lk.lock();
  }
}

static void free_server(sq_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.dmem) (void)hipFree(sl.dmem);
    if (sl.htab) (void)hipHostFree(sl.htab);
  }
  delete s;
}

extern "C" {

int sq_server_create(sq_agent* agent, size_t mem_budget, int max_batch_obs, int n_slots, sq_server** out) {
  if (!agent || !out || max_batch_obs <= 0 || n_slots <= 0 || n_slots > 16 || mem_budget == 0) {
    set_error("bad server arguments (agent, out, max_batch_obs > 0, 1 <= n_slots <= 16, budget > 0)");
    return SQ_EINVAL;
  }
  sq_server* s = new sq_server();
  s->agent = agent;
  s->net = agent_net(agent);
  s->L = agent_layout(agent);
  s->hp = agent_hp(agent);
  s->params = agent_params(agent);
  s->budget = mem_budget;
  s->per_obs = act_bytes_per_obs(s->net);
  s->max_batch = max_batch_obs;
  s->slots.resize(n_slots);
  const sq_dims& d = s->net.d;
  for (Slot& sl : s->slots) {
    Bump b{nullptr};
    plan_act(s->net, max_batch_obs, b, &sl.w);
    b.take<float>((size_t)max_batch_obs * (d.proprio > 0 ? d.proprio : 1));
    b.take<float>((size_t)max_batch_obs * d.action);
    b.take<char>(tables_bytes(max_batch_obs));
    const size_t bytes = b.off + 256;
    if (hipMalloc(&sl.dmem, bytes) != hipSuccess ||
        hipHostMalloc((void**)&sl.htab, tables_bytes(max_batch_obs), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      free_server(s);
      set_error("allocation of %d serving slots of %d observations failed", n_slots, max_batch_obs);
      return SQ_ENOMEM;
    }
    Bump c{(char*)(((uintptr_t)sl.dmem + 255) & ~(uintptr_t)255)};
    plan_act(s->net, max_batch_obs, c, &sl.w);
    sl.prop_stage = c.take<float>((size_t)max_batch_obs * (d.proprio > 0 ? d.proprio : 1));
    sl.act_stage = c.take<float>((size_t)max_batch_obs * d.action);
    sl.dtab = c.take<char>(tables_bytes(max_batch_obs));
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return SQ_OK;
}

int sq_server_submit(sq_server* s, const uint8_t* frames, const float* proprio, int n, int sample,
                     unsigned long long request_id, float* action_out, sq_done_cb cb, void* user) {
  if (!s || (s->net.d.n_conv > 0 && !frames) || !action_out || (s->net.d.proprio > 0 && !proprio) || n <= 0) {
    set_error("bad request arguments");
    return SQ_EINVAL;
  }
  if (n > s->max_batch || (size_t)n * s->per_obs > s->budget) {
    set_error("request of %d observations exceeds the serving limits (max %d, budget %zu bytes)", n, s->max_batch,
              s->budget);
    return SQ_ENOMEM;
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error != SQ_OK) {
      set_error("%s", s->errmsg);
      return s->error;
    }
    s->queue.push_back(Req{frames, proprio, n, sample ? 1 : 0, request_id, action_out, cb, user});
  }
  s->cv.notify_one();
  return SQ_OK;
}

int sq_server_drain(sq_server* s) {
  if (!s) { set_error("server is NULL"); return SQ_EINVAL; }
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.notify_one();
  s->idle.wait(lk, [s] {
    if (!s->queue.empty() || s->firing) return false;
    for (const Slot& sl : s->slots)
      if (sl.busy) return false;
    return true;
  });
  if (s->error != SQ_OK) {
    set_error("%s", s->errmsg);
    return s->error;
  }
  return SQ_OK;
}

int sq_server_destroy(sq_server* s) {
  if (!s) return SQ_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_one();
  s->th.join();
  for (Slot& sl : s->slots) (void)hipStreamSynchronize(sl.st);
  free_server(s);
  return SQ_OK;
}

}  // extern "C"
