// End of one update (Alg. 1 bookkeeping): the update's statistics and the step
// counters.  One 256-thread workgroup; it runs alone, or as the first workgroup of
// the actor's Adam launch, whose update step count was recorded beforehand (so
// the counters this workgroup advances are not read in that launch).
#pragma once
#include "../common.h"

namespace sq {

struct FinishJob {
  const float* loss_row; const float* q_row; const float* tgt_row; const float* logp; const float* qa_row;
  const float* scal; int B; int actor_step; int* ctr; float* stats;
};

// fixed-order tree sum over the 256 threads; valid in every thread
__device__ __forceinline__ float finish_sum256(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

// stats: [0] critic loss (mean over rows of the twin sum), [1] actor loss (0 when
// no actor step), [2] temperature loss, [3] alpha after its step, [4] entropy,
// [5] mean online Q, [6] mean target, [7] 1 if any of them is not finite
__device__ __forceinline__ void finish_block(const FinishJob& f) {
  __shared__ float sh[256];
  const int B = f.B;
  float a = 0.f, q = 0.f, tg = 0.f, pi = 0.f;
  const float alpha_new = f.scal[1];
  for (int i = threadIdx.x; i < B; i += 256) {
    a += f.loss_row[i] + f.loss_row[B + i];
    q += f.q_row[i] + f.q_row[B + i];
    tg += f.tgt_row[i];
    if (f.actor_step) pi += alpha_new * f.logp[i] - f.qa_row[i];
  }
  a = finish_sum256(a, sh);
  q = finish_sum256(q, sh);
  tg = finish_sum256(tg, sh);
  pi = finish_sum256(pi, sh);
  if (threadIdx.x != 0) return;
  float o[8];
  o[0] = a / (float)B;
  o[1] = f.actor_step ? pi / (float)B : 0.f;
  o[2] = f.scal[2];
  o[3] = alpha_new;
  o[4] = f.scal[3];
  o[5] = q / (float)(2 * B);
  o[6] = tg / (float)B;
  int bad = 0;
  for (int i = 0; i < 7; ++i) bad |= !isfinite(o[i]);
  o[7] = bad ? 1.f : 0.f;
  for (int i = 0; i < 8; ++i) f.stats[i] = o[i];
  f.ctr[CTR_U] += 1;
  f.ctr[CTR_TC] += 1;
  f.ctr[CTR_TALPHA] += 1;
  if (f.actor_step) f.ctr[CTR_TA] += 1;
}

}  // namespace sq
