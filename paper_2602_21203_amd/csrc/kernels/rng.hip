// Replay-batch sampling and Gaussian policy noise from Philox4x32-10.
//   replay index  idx[b] = mulhi32(w0, size), counter (u, 0, b, 0), key = seed;
//                 size is read on the device when the replay is a growing ring
//   noise         stream s, element e: Box-Muller on (w0, w1) of counter (u, s, e, 0);
//                 s = 2 feeds the actor sample at s_t, s = 1 the target sample at s_{t+1}
//   act() noise   element e of a request: counter (e, 3, id_lo, id_hi)
#include "../common.h"
#include "philox.h"
#include "sample.h"

namespace sq {

// One thread per (row, item): every thread redraws its row's index (one Philox
// block) and moves one item, so the launch is as wide as the batch's fields.
__global__ __launch_bounds__(256) void k_sample_batch(SampleArgs s) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < sample_items(s.B, s.A, s.S)) sample_item(s, t);
}

SampleArgs sample_args(unsigned long long seed, const int* ctr, int size, const int* dev_size, int B, int A, int S,
                       const float* proprio, const float* next_proprio, const float* action, const float* reward,
                       const uint8_t* done, int* idx, float* eps2B, float* S2, float* Arep, long long ld_arep,
                       float* r, float* d) {
  uint16_t* Arep_h = B > 0 && A > 0 ? twin_of(Arep, (long long)(B - 1) * ld_arep + A) : nullptr;
  return SampleArgs{(unsigned)seed, (unsigned)(seed >> 32), ctr, size, dev_size, B, A, S, proprio, next_proprio,
                    action, reward, done, idx, eps2B, S2, Arep, ld_arep, r, d, Arep_h};
}

int launch_sample_batch(const SampleArgs& s, hipStream_t st) {
  const long long items = sample_items(s.B, s.A, s.S);
  k_sample_batch<<<(unsigned)((items + 255) / 256), 256, 0, st>>>(s);
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
