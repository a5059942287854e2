// encoder_fwd_noalloc: the encoder forward of encoder_fwd for callers that
// cannot allocate (code under graph capture, tight serving loops).  Its scratch
// -- the fused encoder's rearranged weights and the inner layers' activations --
// lives in one file-scope device array of fixed size instead of a workspace.
//
// The array's name is only a host-side stand-in in host code; its device
// address is looked up once per device (with that device current) and kept,
// and only that address is passed to kernels.  Every call on a device shares
// that device's array: calls that overlap on one device (two streams, or two
// threads) race on it and must be ordered by the caller.
#include <mutex>

#include "ops.h"

namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;   // 16 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// the current device's address of `scratch` (looked up on its first use)
int scratch_ptr(char** out) {
  int dev = -1;
  SQ_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    sq::set_error("device %d beyond the %d devices the scratch table holds", dev, kMaxDevices);
    return SQ_EDEVICE;
  }
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      sq::set_error("hipGetSymbolAddress of the encoder scratch failed: %s", hipGetErrorString(e));
      return SQ_EDEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_ptr[dev]);
  return SQ_OK;
}

// the inner layers' activations and the fused path's rearranged weights (the
// last layer is written straight into the caller's feature buffer)
size_t plan(const sq::Net& net, int n, char* base, sq::EncBufs* e, int bf16) {
  const sq_dims& d = net.d;
  sq::Bump b{base};
  *e = sq::EncBufs{};
  for (int i = 0; i + 1 < d.n_conv; ++i)
    e->h[i] = b.take<float>((size_t)n * d.F * net.conv_side[i] * net.conv_side[i]);
  if (sq::encoder_fused_ok(d.C, d.F, d.n_conv, net.side, bf16))
    e->wprep = b.take<float>(sq::encoder_fused_prep_floats(d.C, d.F, d.n_conv));
  return b.off;
}

}  // namespace

using namespace sq;

extern "C" {

int encoder_fwd_noalloc(const sq_dims* dims, sq_prec prec, const float* enc_params, const float* x, int n,
                        float* feat, sq_stream_t stream) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  if (dims->n_conv <= 0) {
    set_error("state-based dims (n_conv = 0) have no frames or encoder");
    return SQ_EINVAL;
  }
  if (n < 0) {
    set_error("n < 0");
    return SQ_EINVAL;
  }
  if (prec != SQ_F32 && prec != SQ_BF16) {
    set_error("unknown precision %d", (int)prec);
    return SQ_EINVAL;
  }
  if (n == 0) return SQ_OK;
  if (!enc_params || !x || !feat) {
    set_error("NULL argument");
    return SQ_EINVAL;
  }
  if ((((uintptr_t)enc_params | (uintptr_t)x | (uintptr_t)feat) & 3u) != 0) {
    set_error("misaligned argument");
    return SQ_EINVAL;
  }
  EncBufs e;
  const size_t need = plan(net, n, nullptr, &e, prec == SQ_BF16);
  if (need > kScratchBytes) {
    set_error("encoder_fwd_noalloc: %d images need %zu scratch bytes, more than the %zu it holds", n, need,
              kScratchBytes);
    return SQ_ENOMEM;
  }
  char* base = nullptr;
  SQ_TRY(scratch_ptr(&base));
  plan(net, n, base, &e, prec == SQ_BF16);
  e.h[dims->n_conv - 1] = feat;
  Layout L;
  make_layout(net, &L);
  return encoder_forward(net, prec == SQ_BF16, enc_params, L, x, n, e, (hipStream_t)stream);
}

int sq_encoder_noalloc_max_images(const sq_dims* dims, int* n) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  if (!n || dims->n_conv <= 0) {
    set_error("NULL n or state-based dims");
    return SQ_EINVAL;
  }
  // the plan grows with n: the largest n whose plan fits (the bfloat16 form's plan,
  // which holds the FP32 form's)
  int lo = 0, hi = 1 << 20;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    EncBufs e;
    if (plan(net, mid, nullptr, &e, 1) <= kScratchBytes) lo = mid; else hi = mid - 1;
  }
  *n = lo;
  return SQ_OK;
}

}  // extern "C"
