// The insert path: a device-resident FIFO replay of squinted transitions.
// Frames are squinted once, when inserted (Alg. 1 downsamples every observation
// as it arrives), and stored as uint8 block means at the squinted size, so an
// update gathers (H/k)(W/k)C bytes per frame instead of H W C.
//
// One launch per insertion: the squint kernel's uint8 mode writes the frames,
// and the first workgroup of each transition's obs image moves its small fields.
// The write position and row count live on the host (insertions are ordered
// by their stream); each insertion also stores the new row count in a device
// int that the update's sampler reads, so a captured update graph keeps
// sampling the whole ring as it grows.
#include <string.h>

#include "ops.h"

using namespace sq;

static int is_capturing(hipStream_t st, bool* cap) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) {
    set_error("hipStreamIsCapturing failed: %s", hipGetErrorString(e));
    return SQ_EDEVICE;
  }
  *cap = cs != hipStreamCaptureStatusNone;
  return SQ_OK;
}

struct sq_ring {
  Net net;
  int cap = 0, pos = 0, size = 0;
  void* mem = nullptr;
  uint8_t *obs = nullptr, *next_obs = nullptr, *done = nullptr;
  float *proprio = nullptr, *next_proprio = nullptr, *action = nullptr, *reward = nullptr;
  int* ctr = nullptr;   // {pos, size} on the device
};

static size_t carve(sq_ring* r, char* base) {
  const int P = r->net.d.proprio > 0 ? r->net.d.proprio : 1, A = r->net.d.action;
  const size_t cap = (size_t)r->cap;
  const size_t frame = (size_t)r->net.side * r->net.side * r->net.d.C;
  Bump b{base};
  r->ctr = b.take<int>(2);
  r->obs = b.take<uint8_t>(cap * frame);
  r->next_obs = b.take<uint8_t>(cap * frame);
  r->proprio = b.take<float>(cap * P);
  r->next_proprio = b.take<float>(cap * P);
  r->action = b.take<float>(cap * A);
  r->reward = b.take<float>(cap);
  r->done = b.take<uint8_t>(cap);
  return b.off + 256;
}

extern "C" {

int sq_ring_create(const sq_dims* dims, int capacity, sq_ring** out) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  if (net.d.n_conv == 0) {
    set_error("state-based dims (n_conv = 0) have no frames to store");
    return SQ_EINVAL;
  }
  if (!out || capacity <= 0) {
    set_error("bad ring arguments (out %p, capacity %d)", (void*)out, capacity);
    return SQ_EINVAL;
  }
  bool cap_now = false;
  SQ_TRY(is_capturing(nullptr, &cap_now));
  if (cap_now) {
    set_error("sq_ring_create allocates and cannot run while the null stream captures");
    return SQ_ECAPTURE;
  }
  sq_ring* r = new sq_ring;
  r->net = net;
  r->cap = capacity;
  const size_t bytes = carve(r, nullptr);
  if (hipMalloc(&r->mem, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of %zu ring bytes failed", bytes);
    delete r;
    return SQ_ENOMEM;
  }
  carve(r, (char*)r->mem);
  // zero rows are valid transitions, so a sampler can never read undefined bytes
  if (hipMemset(r->mem, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    set_error("zero-filling the ring failed");
    (void)hipFree(r->mem);
    delete r;
    return SQ_EDEVICE;
  }
  *out = r;
  return SQ_OK;
}

int sq_ring_destroy(sq_ring* r) {
  if (!r) return SQ_OK;
  if (r->mem) (void)hipFree(r->mem);
  delete r;
  return SQ_OK;
}

int sq_ring_insert(sq_ring* r, const uint8_t* obs, const uint8_t* next_obs, const float* proprio,
                   const float* next_proprio, const float* action, const float* reward, const uint8_t* done, int n,
                   sq_stream_t stream) {
  if (!r) { set_error("ring is NULL"); return SQ_EINVAL; }
  if (n < 0 || n > r->cap) {
    set_error("n = %d outside [0, capacity = %d]", n, r->cap);
    return SQ_EINVAL;
  }
  const sq_dims& d = r->net.d;
  if (n > 0 && (!obs || !next_obs || !action || !reward || !done || (d.proprio > 0 && (!proprio || !next_proprio)))) {
    set_error("NULL argument to sq_ring_insert");
    return SQ_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  bool cap_now = false;
  SQ_TRY(is_capturing(st, &cap_now));
  if (cap_now) {
    set_error("sq_ring_insert keeps the write position on the host and cannot be captured");
    return SQ_ECAPTURE;
  }
  if (n == 0) return SQ_OK;
  const int new_pos = ring_row(r->pos, n, r->cap);
  const int new_size = (int)((long long)r->size + n < r->cap ? r->size + n : r->cap);
  const RingRows f{proprio, next_proprio, action, reward, done, r->proprio, r->next_proprio, r->action, r->reward,
                   r->done, d.proprio, d.action, r->ctr, new_pos, new_size};
  SQ_TRY(launch_squint_insert(obs, next_obs, n, d.H, d.W, d.C, d.k, r->obs, r->next_obs, r->pos, r->cap, f, st));
  r->pos = new_pos;
  r->size = new_size;
  return SQ_OK;
}

int sq_ring_row(int pos, long long i, int capacity, int* row) {
  if (!row || capacity <= 0 || pos < 0 || pos >= capacity || i < 0) {
    set_error("sq_ring_row: need 0 <= pos < capacity, i >= 0 and a row pointer");
    return SQ_EINVAL;
  }
  *row = ring_row(pos, i, capacity);
  return SQ_OK;
}

int sq_ring_view(const sq_ring* r, sq_replay* out) {
  if (!r || !out) { set_error("NULL argument to sq_ring_view"); return SQ_EINVAL; }
  memset(out, 0, sizeof(*out));
  out->obs = r->obs;
  out->next_obs = r->next_obs;
  out->proprio = r->proprio;
  out->next_proprio = r->next_proprio;
  out->action = r->action;
  out->reward = r->reward;
  out->done = r->done;
  out->capacity = r->cap;
  out->size = r->cap;   // fixed, so the view compares equal across inserts; dev_size governs sampling
  out->squinted = 1;
  out->dev_size = r->ctr + 1;
  return SQ_OK;
}

int sq_ring_state(const sq_ring* r, int* pos, int* size) {
  if (!r || !pos || !size) { set_error("NULL argument to sq_ring_state"); return SQ_EINVAL; }
  *pos = r->pos;
  *size = r->size;
  return SQ_OK;
}

int sq_ring_copy_out(const sq_ring* r, int field, int row0, int n, void* dst, sq_stream_t stream) {
  if (!r || (!dst && n > 0)) { set_error("NULL argument to sq_ring_copy_out"); return SQ_EINVAL; }
  if (row0 < 0 || n < 0 || (long long)row0 + n > r->cap) {
    set_error("rows [%d, %d + %d) outside [0, %d)", row0, row0, n, r->cap);
    return SQ_EINVAL;
  }
  const int P = r->net.d.proprio, A = r->net.d.action;
  const size_t frame = (size_t)r->net.side * r->net.side * r->net.d.C;
  const void* src;
  size_t row_bytes;
  switch (field) {
    case SQ_RING_OBS: src = r->obs; row_bytes = frame; break;
    case SQ_RING_NEXT_OBS: src = r->next_obs; row_bytes = frame; break;
    case SQ_RING_PROPRIO: src = r->proprio; row_bytes = sizeof(float) * P; break;
    case SQ_RING_NEXT_PROPRIO: src = r->next_proprio; row_bytes = sizeof(float) * P; break;
    case SQ_RING_ACTION: src = r->action; row_bytes = sizeof(float) * A; break;
    case SQ_RING_REWARD: src = r->reward; row_bytes = sizeof(float); break;
    case SQ_RING_DONE: src = r->done; row_bytes = 1; break;
    default: set_error("unknown ring field %d", field); return SQ_EINVAL;
  }
  if (n == 0 || row_bytes == 0) return SQ_OK;
  const hipError_t e = hipMemcpyAsync(dst, (const char*)src + (size_t)row0 * row_bytes, (size_t)n * row_bytes,
                                      hipMemcpyDefault, (hipStream_t)stream);
  if (e != hipSuccess) {
    set_error("hipMemcpyAsync from the ring failed: %s", hipGetErrorString(e));
    return SQ_EDEVICE;
  }
  return SQ_OK;
}

}  // extern "C"
