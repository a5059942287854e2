// FIFO replay ring of squinted transitions (Alg. 1 stores the downsampled
// observation pair with proprio, action and reward; the buffer is a plain FIFO
// held on the GPU, Sec. V Replay Buffer Size).  The frames go through the squint
// kernel's uint8 mode; this file moves the small per-transition fields.
#include "../common.h"

namespace sq {

// One thread per (transition, item): items are the 2P proprio values, A action
// values, the reward and the done flag of a transition.  Thread 0 also stores the
// ring's counters after this insertion (nothing in this launch reads them).
__global__ __launch_bounds__(256) void k_ring_fields(const float* __restrict__ proprio,
                                                     const float* __restrict__ next_proprio,
                                                     const float* __restrict__ action,
                                                     const float* __restrict__ reward,
                                                     const uint8_t* __restrict__ done, int n, int P, int A,
                                                     float* __restrict__ r_proprio, float* __restrict__ r_next,
                                                     float* __restrict__ r_action, float* __restrict__ r_reward,
                                                     uint8_t* __restrict__ r_done, int pos, int cap,
                                                     int* __restrict__ ctr, int new_pos, int new_size) {
  const int W = 2 * P + A + 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ctr[0] = new_pos;
    ctr[1] = new_size;
  }
  if (t >= (long long)n * W) return;
  const int i = (int)(t / W), it = (int)(t - (long long)i * W);
  const long long row = (pos + i) % cap;
  if (it < P) r_proprio[row * P + it] = proprio[(long long)i * P + it];
  else if (it < 2 * P) r_next[row * P + it - P] = next_proprio[(long long)i * P + it - P];
  else if (it < 2 * P + A) r_action[row * A + it - 2 * P] = action[(long long)i * A + it - 2 * P];
  else if (it == 2 * P + A) r_reward[row] = reward[i];
  else r_done[row] = done[i];
}

int launch_ring_fields(const float* proprio, const float* next_proprio, const float* action, const float* reward,
                       const uint8_t* done, int n, int P, int A, float* r_proprio, float* r_next_proprio,
                       float* r_action, float* r_reward, uint8_t* r_done, int pos, int cap, int* ctr, int new_pos,
                       int new_size, hipStream_t st) {
  const long long items = (long long)n * (2 * P + A + 2);
  const unsigned blocks = (unsigned)((items + 255) / 256);
  k_ring_fields<<<blocks > 0 ? blocks : 1, 256, 0, st>>>(proprio, next_proprio, action, reward, done, n, P, A,
                                                          r_proprio, r_next_proprio, r_action, r_reward, r_done, pos,
                                                          cap, ctr, new_pos, new_size);
  return launch_status("ring_fields");
}

}  // namespace sq
