// bfloat16 copies ("twins") of FP32 operand buffers.
//
// In the bfloat16 mode every linear-layer product rounds its operands to
// bfloat16 before the matrix cores.  An owner (the agent) may register, for an
// FP32 buffer, a uint16 buffer of the same element count; every kernel that
// writes the FP32 buffer then also writes the rounded value at the same element
// offset of the twin, and a product whose operands both have twins reads the
// twins (half the bytes, no conversion) instead.  Rounding once at the producer
// or at the consumer gives the same bfloat16 value, so results are identical.
// Where every reader of a buffer reads its twin, the owner may also drop the
// FP32 values (fp32_drop_register): the producers then write the twin only, and
// a product that would have to read the FP32 values fails instead of reading
// stale ones.
#include <atomic>
#include <mutex>
#include <vector>

#include "common.h"

namespace sq {

namespace {
struct TwinRange {
  const void* owner; const float* f; long long n; uint16_t* h;
};
std::mutex g_mu;
std::vector<TwinRange> g_ranges;
std::vector<TwinRange> g_dropped;   // FP32 ranges whose values are no longer kept (h unused)
int g_enabled = 1;
std::atomic<long long> g_products{0};
}  // namespace

void note_copy_product() { g_products.fetch_add(1, std::memory_order_relaxed); }
long long copy_products() { return g_products.load(std::memory_order_relaxed); }

int twins_enabled() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_enabled;
}

int set_twins_enabled(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int was = g_enabled;
  g_enabled = on ? 1 : 0;
  return was;
}

void twin_register(const void* owner, const float* f, long long n, uint16_t* h) {
  if (!f || !h || n <= 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_ranges.push_back(TwinRange{owner, f, n, h});
}

void fp32_drop_register(const void* owner, const float* f, long long n) {
  if (!f || n <= 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_dropped.push_back(TwinRange{owner, f, n, nullptr});
}

void twin_unregister(const void* owner) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (std::vector<TwinRange>* v : {&g_ranges, &g_dropped}) {
    std::vector<TwinRange> keep;
    for (const TwinRange& r : *v)
      if (r.owner != owner) keep.push_back(r);
    v->swap(keep);
  }
}

bool fp32_dropped(const float* f) {
  if (!f) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  const uintptr_t a = (uintptr_t)f;
  for (const TwinRange& r : g_dropped) {
    const uintptr_t b = (uintptr_t)r.f;
    if (a >= b && a < b + (uintptr_t)r.n * sizeof(float)) return true;
  }
  return false;
}

uint16_t* twin_of(const float* f, long long n) {
  if (!f || n <= 0) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  const uintptr_t a = (uintptr_t)f, e = a + (uintptr_t)n * sizeof(float);
  for (const TwinRange& r : g_ranges) {
    const uintptr_t b = (uintptr_t)r.f;
    if (a >= b && e <= b + (uintptr_t)r.n * sizeof(float)) return r.h + (f - r.f);
  }
  return nullptr;
}

}  // namespace sq
