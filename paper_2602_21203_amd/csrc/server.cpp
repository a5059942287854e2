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

#include <algorithm>
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
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // device start / end of the slot's batch (timing)
  void* dmem = nullptr;
  char* htab = nullptr;
  char* dtab = nullptr;
  ActBufs w;
  float* prop_stage = nullptr;
  float* act_stage = nullptr;
  std::vector<Req> batch;
  bool busy = false;
  bool finished = false;   // set by the stream's host function when the batch is done
  size_t bytes = 0;
  sq_server* srv = nullptr;
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
  bool hold = false;   // admissions paused (sq_server_hold)
  size_t firing = 0;   // completions whose callbacks are running
  int error = SQ_OK;
  char errmsg[256] = {0};
  // counters (under mu)
  sq_server_stats st{};
  hipEvent_t ref = nullptr;                        // time origin of the device intervals
  std::vector<std::pair<double, double>> spans;    // device [start, end] of every batch, seconds
};

// host function enqueued after each batch: marks the slot finished and wakes
// the scheduler (no HIP calls here)
static void batch_done(void* arg) {
  Slot* sl = static_cast<Slot*>(arg);
  sq_server* s = sl->srv;
  {
    std::lock_guard<std::mutex> g(s->mu);
    sl->finished = true;
  }
  s->cv.notify_one();
}

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
  SQ_TRY_HIP(hipEventRecord(sl.ev0, st));
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
  SQ_TRY_HIP(hipEventRecord(sl.ev1, st));
  SQ_TRY_HIP(hipLaunchHostFunc(st, batch_done, &sl));
  return SQ_OK;
}

// The scheduler thread owns the slots' batches; the mutex guards the queue, the
// slots' busy / finished flags, the memory in flight and the counters.  Launches,
// event reads and completion callbacks run with the mutex released.
static void scheduler(sq_server* s) {
  std::vector<Req> done;
  std::vector<Slot*> to_launch;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // completions: batches whose host function has run
    std::vector<Slot*> fin;
    for (Slot& sl : s->slots)
      if (sl.busy && sl.finished) fin.push_back(&sl);
    if (!fin.empty()) {
      lk.unlock();
      std::vector<std::pair<double, double>> spans;
      int err = SQ_OK;
      char msg[200] = {0};
      for (Slot* sl : fin) {
        float t0 = 0.f, t1 = 0.f;
        const hipError_t e0 = hipEventElapsedTime(&t0, s->ref, sl->ev0);
        const hipError_t e1 = hipEventElapsedTime(&t1, s->ref, sl->ev1);
        if (e0 != hipSuccess || e1 != hipSuccess) {
          err = SQ_EDEVICE;
          snprintf(msg, sizeof(msg), "act batch failed: %s", hipGetErrorString(e0 != hipSuccess ? e0 : e1));
        } else {
          spans.emplace_back(1e-3 * t0, 1e-3 * t1);
        }
        for (const Req& r : sl->batch) done.push_back(r);
      }
      lk.lock();
      for (Slot* sl : fin) {
        sl->batch.clear();
        sl->busy = false;
        sl->finished = false;
        s->in_flight -= sl->bytes;
        sl->bytes = 0;
      }
      s->spans.insert(s->spans.end(), spans.begin(), spans.end());
      if (err != SQ_OK && s->error == SQ_OK) {
        s->error = err;
        snprintf(s->errmsg, sizeof(s->errmsg), "%s", msg);
      }
    }
    // admissions: FIFO, fuse every head request that fits
    int busy_now = 0;
    for (Slot& sl : s->slots) busy_now += sl.busy;
    for (Slot& sl : s->slots) {
      if (s->hold || sl.busy || s->queue.empty()) continue;
      int rows = 0, nreq = 0;
      while (!s->queue.empty()) {
        const Req& q = s->queue.front();
        const size_t need = (size_t)(rows + q.n) * s->per_obs;
        if (rows + q.n > s->max_batch || s->in_flight + need > s->budget) break;
        rows += q.n;
        ++nreq;
        sl.batch.push_back(q);
        s->queue.pop_front();
      }
      if (rows == 0) break;   // the head does not fit yet: wait for completions
      sl.bytes = (size_t)rows * s->per_obs;
      s->in_flight += sl.bytes;
      sl.busy = true;
      sl.finished = false;
      ++busy_now;
      s->st.batches += 1;
      s->st.requests += nreq;
      s->st.rows += rows;
      if (nreq > 1) s->st.fused_batches += 1;
      if (nreq > s->st.max_requests_per_batch) s->st.max_requests_per_batch = nreq;
      if (busy_now > s->st.max_slots_busy) s->st.max_slots_busy = busy_now;
      to_launch.push_back(&sl);
    }
    if (!to_launch.empty() || !done.empty()) {
      std::vector<Req> fire;
      fire.swap(done);
      std::vector<Slot*> launch;
      launch.swap(to_launch);
      s->firing = fire.size();
      lk.unlock();
      int err = SQ_OK;
      char msg[256] = {0};
      for (Slot* sl : launch)
        if (launch_batch(s, *sl) != SQ_OK) {
          err = SQ_EDEVICE;
          snprintf(msg, sizeof(msg), "%s", sq_last_error());
          (void)hipStreamSynchronize(sl->st);
          batch_done(sl);   // nothing more will complete on this slot's stream
        }
      const double t = now_s();
      for (const Req& r : fire)
        if (r.cb) r.cb(r.id, t, r.user);
      lk.lock();
      s->firing = 0;
      if (err != SQ_OK && s->error == SQ_OK) {
        s->error = err;
        snprintf(s->errmsg, sizeof(s->errmsg), "%s", msg);
      }
      continue;
    }
    bool any_busy = false;
    for (const Slot& sl : s->slots) any_busy |= sl.busy;
    if (!any_busy && s->queue.empty()) {
      s->idle.notify_all();
      if (s->stop) break;
    }
    // sleep until a submit, a completion, a hold change or the stop
    s->cv.wait(lk);
  }
}

static void free_server(sq_server* s) {
  if (s->ref) (void)hipEventDestroy(s->ref);
  for (Slot& sl : s->slots) {
    if (sl.ev0) (void)hipEventDestroy(sl.ev0);
    if (sl.ev1) (void)hipEventDestroy(sl.ev1);
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
        hipEventCreate(&sl.ev0) != hipSuccess || hipEventCreate(&sl.ev1) != hipSuccess) {
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
  for (Slot& sl : s->slots) sl.srv = s;
  if (hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, s->slots[0].st) != hipSuccess ||
      hipEventSynchronize(s->ref) != hipSuccess) {
    free_server(s);
    set_error("creating the server's reference event failed");
    return SQ_EDEVICE;
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

int sq_server_hold(sq_server* s, int hold) {
  if (!s) { set_error("server is NULL"); return SQ_EINVAL; }
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->hold = hold != 0;
  }
  s->cv.notify_one();
  return SQ_OK;
}

int sq_server_get_stats(sq_server* s, sq_server_stats* out) {
  if (!s || !out) { set_error("NULL argument to sq_server_get_stats"); return SQ_EINVAL; }
  std::vector<std::pair<double, double>> spans;
  {
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    spans = s->spans;
  }
  // union of the batches' device intervals, and whether any two overlapped
  std::sort(spans.begin(), spans.end());
  double busy = 0.0, cur0 = 0.0, cur1 = -1.0, first = 0.0, last = 0.0;
  long long overlaps = 0;
  for (size_t i = 0; i < spans.size(); ++i) {
    const auto& sp = spans[i];
    if (i == 0) first = sp.first;
    if (sp.second > last) last = sp.second;
    if (sp.first < cur1) {
      ++overlaps;
      if (sp.second > cur1) cur1 = sp.second;
    } else {
      if (cur1 > cur0) busy += cur1 - cur0;
      cur0 = sp.first;
      cur1 = sp.second;
    }
  }
  if (cur1 > cur0) busy += cur1 - cur0;
  out->device_busy_s = busy;
  out->device_span_s = spans.empty() ? 0.0 : last - first;
  out->overlapped_batches = overlaps;
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
