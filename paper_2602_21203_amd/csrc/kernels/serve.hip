// Small per-row kernels of the continuous-batching act() server: requests of
// one fused launch live in separate caller buffers, reached through per-row
// pointer tables.
#include "../common.h"
#include "philox.h"

namespace sq {

__global__ void k_gather_rows(const float* const* __restrict__ src, int width, int n, float* __restrict__ dst) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * width) return;
  const int r = (int)(e / width), j = (int)(e - (long long)r * width);
  dst[e] = src[r][j];
}

int gather_rows(const float* const* src, int width, int n, float* dst, hipStream_t st) {
  if (n <= 0 || width <= 0) return SQ_OK;
  k_gather_rows<<<cdiv((long long)n * width, 256), 256, 0, st>>>(src, width, n, dst);
  return launch_status("gather_rows");
}

__global__ void k_scatter_rows(const float* __restrict__ src, int width, int n, float* const* __restrict__ dst) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * width) return;
  const int r = (int)(e / width), j = (int)(e - (long long)r * width);
  dst[r][j] = src[e];
}

int scatter_rows(const float* src, int width, int n, float* const* dst, hipStream_t st) {
  if (n <= 0 || width <= 0) return SQ_OK;
  k_scatter_rows<<<cdiv((long long)n * width, 256), 256, 0, st>>>(src, width, n, dst);
  return launch_status("scatter_rows");
}

// noise of row r: element e = rows[r] * A + d of request ids[r], counter
// (e, 3, id_lo, id_hi) -- the same value act() draws for that request alone;
// rows that ask for the mean action get eps = 0 (tanh(mu + sigma * 0) = tanh(mu))
__global__ void k_act_noise_rows(unsigned k0, unsigned k1, const unsigned long long* __restrict__ ids,
                                 const int* __restrict__ rows, const int* __restrict__ sample, int n, int A,
                                 float* __restrict__ eps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * A) return;
  const int r = e / A, d = e - r * A;
  if (!sample[r]) {
    eps[e] = 0.f;
    return;
  }
  const unsigned long long id = ids[r];
  const P4 w = philox10(P4{(unsigned)(rows[r] * A + d), 3u, (unsigned)id, (unsigned)(id >> 32)}, k0, k1);
  eps[e] = box_muller(w.x, w.y);
}

int act_noise_rows(unsigned long long seed, const unsigned long long* ids, const int* rows, const int* sample, int n,
                   int A, float* eps, hipStream_t st) {
  if (n <= 0) return SQ_OK;
  k_act_noise_rows<<<cdiv((long long)n * A, 256), 256, 0, st>>>((unsigned)seed, (unsigned)(seed >> 32), ids, rows,
                                                                 sample, n, A, eps);
  return launch_status("act_noise_rows");
}

}  // namespace sq
