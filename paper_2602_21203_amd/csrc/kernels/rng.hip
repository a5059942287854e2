// Replay-batch sampling and Gaussian policy noise from Philox4x32-10.
//   replay index  idx[b] = mulhi32(w0, size), counter (u, 0, b, 0), key = seed;
//                 size is read on the device when the replay is a growing ring
//   noise         stream s, element e: Box-Muller on (w0, w1) of counter (u, s, e, 0);
//                 s = 2 feeds the actor sample at s_t, s = 1 the target sample at s_{t+1}
//   act() noise   element e of a request: counter (e, 3, id_lo, id_hi)
#include "../common.h"
#include "philox.h"

namespace sq {

// One thread per (row, item): every thread redraws its row's index (one Philox
// block) and moves one item -- a proprio value of s or s', an action value, one
// of the row's 2 x A noise values, the reward or the done flag -- so the launch
// is as wide as the batch's fields.  eps2B rows [0, B) = stream 2, rows [B, 2B) =
// stream 1.
__global__ __launch_bounds__(256) void k_sample_batch(unsigned k0, unsigned k1, const int* __restrict__ ctr,
                                                      int size, const int* __restrict__ dev_size, int B, int A,
                                                      int S,
                                                      const float* __restrict__ proprio,
                                                      const float* __restrict__ next_proprio,
                                                      const float* __restrict__ action,
                                                      const float* __restrict__ reward,
                                                      const uint8_t* __restrict__ done, int* __restrict__ idx,
                                                      float* __restrict__ eps2B, float* __restrict__ S2,
                                                      float* __restrict__ Arep, float* __restrict__ r,
                                                      float* __restrict__ d) {
  const int W = 2 * S + 3 * A + 2;   // items per row
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * W) return;
  const int b = (int)(t / W), it = (int)(t - (long long)b * W);
  const unsigned u = (unsigned)ctr[CTR_U];
  if (it < 3 * A + 2 && it >= A && it < 3 * A) {   // noise: no replay access
    const int j = (it - A) % A;
    const unsigned s = it < 2 * A ? 2u : 1u;
    const P4 g = philox10(P4{u, s, (unsigned)(b * A + j), 0u}, k0, k1);
    eps2B[(long long)(s == 2u ? b : B + b) * A + j] = box_muller(g.x, g.y);
    return;
  }
  const P4 w = philox10(P4{u, 0u, (unsigned)b, 0u}, k0, k1);
  const int row = (int)__umulhi(w.x, (unsigned)(dev_size ? *dev_size : size));
  if (it < A) {
    Arep[(long long)b * A + it] = action[(long long)row * A + it];
  } else if (it == 3 * A) {
    r[b] = reward[row];
    idx[b] = row;
  } else if (it == 3 * A + 1) {
    d[b] = done[row] ? 1.0f : 0.0f;
  } else {
    const int j = it - (3 * A + 2);
    if (j < S) S2[(long long)b * S + j] = proprio[(long long)row * S + j];
    else S2[(long long)(B + b) * S + (j - S)] = next_proprio[(long long)row * S + (j - S)];
  }
}

int launch_sample_batch(unsigned long long seed, const int* ctr, int size, const int* dev_size, int B, int A, int S,
                        const float* proprio, const float* next_proprio, const float* action,
                        const float* reward, const uint8_t* done, int* idx, float* eps2B, float* S2,
                        float* Arep, float* r, float* d, hipStream_t st) {
  const long long items = (long long)B * (2 * S + 3 * A + 2);
  k_sample_batch<<<(unsigned)((items + 255) / 256), 256, 0, st>>>((unsigned)seed, (unsigned)(seed >> 32), ctr, size,
                                                                  dev_size, B, A, S, proprio, next_proprio, action, reward,
                                                                  done, idx, eps2B, S2, Arep, r, d);
  return launch_status("sample_batch");
}

__global__ void k_indices(unsigned k0, unsigned k1, unsigned u, int size, int n, int* __restrict__ idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const P4 w = philox10(P4{u, 0u, (unsigned)b, 0u}, k0, k1);
  idx[b] = (int)__umulhi(w.x, (unsigned)size);
}

int launch_indices(unsigned long long seed, unsigned update, int size, int n, int* idx, hipStream_t st) {
  k_indices<<<cdiv(n, 256), 256, 0, st>>>((unsigned)seed, (unsigned)(seed >> 32), update, size, n, idx);
  return launch_status("indices");
}

__global__ void k_gaussian(unsigned k0, unsigned k1, unsigned c0, unsigned c1, unsigned c3_lo,
                           unsigned c3_hi, int mode, int n, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  // mode 0: counter (c0, c1, e, 0); mode 1 (act noise): counter (e, c1, c3_lo, c3_hi)
  const P4 c = mode == 0 ? P4{c0, c1, (unsigned)e, 0u} : P4{(unsigned)e, c1, c3_lo, c3_hi};
  const P4 w = philox10(c, k0, k1);
  out[e] = box_muller(w.x, w.y);
}

int launch_gaussian(unsigned long long seed, unsigned update, unsigned stream_id, int n, float* out,
                    hipStream_t st) {
  k_gaussian<<<cdiv(n, 256), 256, 0, st>>>((unsigned)seed, (unsigned)(seed >> 32), update, stream_id, 0u,
                                           0u, 0, n, out);
  return launch_status("gaussian");
}

int launch_act_noise(unsigned long long seed, unsigned long long request_id, int rows, int A, float* out,
                     hipStream_t st) {
  const int n = rows * A;
  k_gaussian<<<cdiv(n, 256), 256, 0, st>>>((unsigned)seed, (unsigned)(seed >> 32), 0u, 3u,
                                           (unsigned)request_id, (unsigned)(request_id >> 32), 1, n, out);
  return launch_status("act_noise");
}

}  // namespace sq
