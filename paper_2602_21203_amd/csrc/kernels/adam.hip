// Adam with bias correction, fused with the target-critic EMA (Alg. 1 target
// update) and an optional bfloat16 copy of the new parameters.  One flat launch
// covers a whole optimiser group (encoder + critic, or actor).
#include <math.h>

#include "../common.h"
#include "bf16.h"

namespace sq {

// the packed position of flat index i (relative to the optimiser's range), or -1
__device__ __forceinline__ long long pack_pos(const PackArgs& pk, long long i, int* critic) {
  const long long gi = i + pk.p_begin;
  for (int s = 0; s < pk.n; ++s) {
    const PackSeg& q = pk.seg[s];
    const long long loc = gi - q.src;
    if (loc >= 0 && loc < (long long)q.rows * q.cols) {
      const long long r = loc / q.cols;
      *critic = q.critic;
      return q.dst + r * q.ldp + (loc - r * q.cols);
    }
  }
  return -1;
}

// Each workgroup updates 256 * kAdamPer consecutive parameters.  The packed
// segment holding the workgroup's first parameter is found once; parameters of
// that segment map to their packed position with one division, the rare others
// (a workgroup straddling a segment boundary) search the table.
constexpr int kAdamPer = 4;

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long long n,
                                              float lr, float b1, float b2, float eps,
                                              const int* __restrict__ step, float* __restrict__ ema,
                                              long long ema_begin, float rho, uint16_t* __restrict__ shadow,
                                              PackArgs pk) {
  const float t = (float)(*step + 1);
  const float bc1 = 1.f - powf(b1, t);
  const float bc2 = 1.f - powf(b2, t);
  const long long b0 = (long long)blockIdx.x * 256 * kAdamPer;
  int s0 = -1;
  for (int s = 0; s < pk.n; ++s) {
    const long long loc = b0 + pk.p_begin - pk.seg[s].src;
    if (loc >= 0 && loc < (long long)pk.seg[s].rows * pk.seg[s].cols) { s0 = s; break; }
  }
#pragma unroll
  for (int u = 0; u < kAdamPer; ++u) {
    const long long i = b0 + u * 256 + threadIdx.x;
    if (i >= n) break;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    float ei = 0.f;
    if (ema && i >= ema_begin) {
      float* e = ema + (i - ema_begin);
      ei = rho * *e + (1.f - rho) * pi;
      *e = ei;
    }
    if (shadow) shadow[i] = bf16_bits(pi);
    if (pk.n) {
      int critic = 0;
      long long d = -1;
      if (s0 >= 0) {
        const PackSeg& q = pk.seg[s0];
        const long long loc = i + pk.p_begin - q.src;
        if (loc < (long long)q.rows * q.cols) {
          const unsigned r = (unsigned)loc / (unsigned)q.cols;
          d = q.dst + (long long)r * q.ldp + (loc - (long long)r * q.cols);
          critic = q.critic;
        }
      }
      if (d < 0) d = pack_pos(pk, i, &critic);
      if (d >= 0) {
        pk.pack[d] = pi;
        if (critic && pk.tpack && ema && i >= ema_begin) pk.tpack[d] = ei;
      }
    }
  }
}

int adam(float* p, const float* g, float* m, float* v, long long n, const sq_hparams* hp, const int* step,
         float* ema_target, long long ema_begin, uint16_t* shadow, const PackArgs* pk, hipStream_t st) {
  if (n <= 0) return SQ_OK;
  const long long blocks = (n + 256 * kAdamPer - 1) / (256 * kAdamPer);
  PackArgs none{};
  k_adam<<<(unsigned)blocks, 256, 0, st>>>(p, g, m, v, n, hp->lr, hp->beta1, hp->beta2, hp->adam_eps, step,
                                           ema_target, ema_begin, hp->rho, shadow, pk ? *pk : none);
  return launch_status("adam");
}

// rows of every packed segment; padding columns are written as zero
__global__ void k_pack(PackArgs pk, const float* __restrict__ params, const float* __restrict__ target,
                       long long critic_begin) {
  const PackSeg q = pk.seg[blockIdx.y];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)q.rows * q.ldp;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / q.ldp, c = e - r * q.ldp;
    const bool in = c < q.cols;
    pk.pack[q.dst + e] = in ? params[q.src + r * q.cols + c] : 0.f;
    if (q.critic && pk.tpack) pk.tpack[q.dst + e] = in ? target[q.src - critic_begin + r * q.cols + c] : 0.f;
  }
}

int pack_weights(const Layout& L, const float* params, const float* target, float* pack, float* tpack,
                 hipStream_t st) {
  PackArgs pk{};
  pk.n = L.n_pack;
  for (int i = 0; i < L.n_pack; ++i) pk.seg[i] = L.pack[i];
  pk.pack = pack;
  pk.tpack = target ? tpack : nullptr;
  k_pack<<<dim3(64, L.n_pack), 256, 0, st>>>(pk, params, target, L.critic_begin);
  return launch_status("pack_weights");
}

}  // namespace sq
