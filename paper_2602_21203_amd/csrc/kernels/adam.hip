// Adam with bias correction, fused with the target-critic EMA (Alg. 1 target
// update) and an optional bfloat16 copy of the new parameters.  One flat launch
// covers a whole optimiser group (encoder + critic, or actor).
#include <math.h>

#include "../common.h"
#include "bf16.h"

namespace sq {

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long long n,
                                              float lr, float b1, float b2, float eps,
                                              const int* __restrict__ step, float* __restrict__ ema,
                                              long long ema_begin, float rho, uint16_t* __restrict__ shadow) {
  const float t = (float)(*step + 1);
  const float bc1 = 1.f - powf(b1, t);
  const float bc2 = 1.f - powf(b2, t);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (ema && i >= ema_begin) {
      float* e = ema + (i - ema_begin);
      *e = rho * *e + (1.f - rho) * pi;
    }
    if (shadow) shadow[i] = bf16_bits(pi);
  }
}

int adam(float* p, const float* g, float* m, float* v, long long n, const sq_hparams* hp, const int* step,
         float* ema_target, long long ema_begin, uint16_t* shadow, hipStream_t st) {
  if (n <= 0) return SQ_OK;
  long long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  k_adam<<<(int)blocks, 256, 0, st>>>(p, g, m, v, n, hp->lr, hp->beta1, hp->beta2, hp->adam_eps, step, ema_target,
                                      ema_begin, hp->rho, shadow);
  return launch_status("adam");
}

}  // namespace sq
