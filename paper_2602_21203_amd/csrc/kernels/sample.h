// One item of the update's minibatch draw (Alg. 1: sample a minibatch from the
// replay buffer; uniform with replacement, Philox4x32-10 keyed by (seed, u)).
// Items of row b: A replayed action values (row b of Arep, stride ld_arep), 2A policy-noise values (stream 2 for
// the sample at s_t, stream 1 for s_{t+1}), the reward, the done flag, and the 2S
// proprio values of s and s'.  Shared by the standalone sampling launch and the
// squint launch that samples in extra workgroups; both give identical results.
#pragma once
#include "../common.h"
#include "bf16.h"
#include "philox.h"

namespace sq {

struct SampleArgs {
  unsigned k0, k1; const int* ctr; int size; const int* dev_size; int B, A, S;
  const float* proprio; const float* next_proprio; const float* action; const float* reward;
  const uint8_t* done;
  int* idx; float* eps2B; float* S2; float* Arep; long long ld_arep; float* r; float* d;
  uint16_t* Arep_h;   // bfloat16 copy of Arep's buffer (nullable)
};

__host__ __device__ inline long long sample_items(int B, int A, int S) { return (long long)B * (2 * S + 3 * A + 2); }

// replay row of batch row b: mulhi32(w0, size) of counter (u, 0, b, 0)
__device__ __forceinline__ int sample_row(const SampleArgs& s, int b) {
  const unsigned u = (unsigned)s.ctr[CTR_U];
  const P4 w = philox10(P4{u, 0u, (unsigned)b, 0u}, s.k0, s.k1);
  return (int)__umulhi(w.x, (unsigned)(s.dev_size ? *s.dev_size : s.size));
}

__device__ __forceinline__ void sample_item(const SampleArgs& s, long long t) {
  const int A = s.A, S = s.S, B = s.B;
  const int W = 2 * S + 3 * A + 2;   // items per row
  const int b = (int)(t / W), it = (int)(t - (long long)b * W);
  if (it >= A && it < 3 * A) {   // noise: no replay access
    const unsigned u = (unsigned)s.ctr[CTR_U];
    const int j = (it - A) % A;
    const unsigned st = it < 2 * A ? 2u : 1u;
    const P4 g = philox10(P4{u, st, (unsigned)(b * A + j), 0u}, s.k0, s.k1);
    s.eps2B[(long long)(st == 2u ? b : B + b) * A + j] = box_muller(g.x, g.y);
    return;
  }
  const int row = sample_row(s, b);
  if (it < A) {
    const float a = s.action[(long long)row * A + it];
    s.Arep[(long long)b * s.ld_arep + it] = a;
    if (s.Arep_h) s.Arep_h[(long long)b * s.ld_arep + it] = bf16_bits(a);
  } else if (it == 3 * A) {
    s.r[b] = s.reward[row];
    s.idx[b] = row;
  } else if (it == 3 * A + 1) {
    s.d[b] = s.done[row] ? 1.0f : 0.0f;
  } else {
    const int j = it - (3 * A + 2);
    if (j < S) s.S2[(long long)b * S + j] = s.proprio[(long long)row * S + j];
    else s.S2[(long long)(B + b) * S + (j - S)] = s.next_proprio[(long long)row * S + (j - S)];
  }
}

}  // namespace sq
