// Resolution squinting: gather replay frames and take k x k block means.
// A workgroup owns `ry` output rows of one image: it streams the k*ry source pixel
// rows (contiguous in the HWC frame) into LDS with 16-byte loads, then each thread
// forms exact integer block sums S from LDS and emits either the network input
// x = S / (255 k^2) - 0.5 (CHW, FP32 or bfloat16) or, when frames are squinted at
// insertion, the uint8 block mean (HWC, nearest with ties to even) into a FIFO ring.
#include "../common.h"
#include "bf16.h"
#include "sample.h"

namespace sq {

// rounded block mean: nearest integer to s / kk, ties to even (s >= 0)
__device__ __forceinline__ unsigned mean_u8(int s, int kk) {
  const int q = s / kk, r = s - q * kk;
  return (unsigned)(q + ((2 * r > kk) || (2 * r == kk && (q & 1))));
}

// one output value of image img at channel c, pixel (y, x) of the side x side grid
__device__ __forceinline__ void emit(const SqDst& d, int img, int nsplit, int C, int side, int c, int y, int x, int s,
                                     int kk, float scale) {
  if (d.mode == kSqU8) {
    const bool second = img >= nsplit;
    const int row = ring_row(d.pos, second ? img - nsplit : img, d.cap);
    uint8_t* base = reinterpret_cast<uint8_t*>(second ? d.out1 : d.out) + (long long)row * side * side * C;
    base[((long long)y * side + x) * C + c] = (uint8_t)mean_u8(s, kk);
    return;
  }
  const float v = (float)s / scale - 0.5f;
  const long long oi = (long long)img * d.row_stride + ((long long)c * side + y) * side + x;
  if (d.mode == kSqBF16)
    reinterpret_cast<uint16_t*>(d.out)[oi] = bf16_bits(v);
  else
    reinterpret_cast<float*>(d.out)[oi] = v;
}

// a transition's small fields into its ring row, by the first workgroup of its
// obs image; image 0 also stores the ring's counters (nothing in the launch reads them)
__device__ __forceinline__ void ring_fields(const SqDst& d, int i) {
  const RingRows& f = d.f;
  const int W = 2 * f.P + f.A + 2;
  const long long row = ring_row(d.pos, i, d.cap);
  for (int it = threadIdx.x; it < W; it += blockDim.x) {
    if (it < f.P) f.r_proprio[row * f.P + it] = f.proprio[(long long)i * f.P + it];
    else if (it < 2 * f.P) f.r_next[row * f.P + it - f.P] = f.next_proprio[(long long)i * f.P + it - f.P];
    else if (it < 2 * f.P + f.A) f.r_action[row * f.A + it - 2 * f.P] = f.action[(long long)i * f.A + it - 2 * f.P];
    else if (it == 2 * f.P + f.A) f.r_reward[row] = f.reward[i];
    else f.r_done[row] = f.done[i];
  }
  if (i == 0 && threadIdx.x == 0) {
    f.ctr[0] = f.new_pos;
    f.ctr[1] = f.new_size;
  }
}

__device__ __forceinline__ const uint8_t* source_row(const uint8_t* src0, const uint8_t* src1, const int* idx,
                                                     const uint8_t* const* row_ptrs, int nsplit, int img,
                                                     long long frame_bytes) {
  if (row_ptrs) return row_ptrs[img];
  if (img < nsplit) return src0 + (idx ? idx[img] : img) * frame_bytes;
  return src1 + (idx ? idx[img - nsplit] : img - nsplit) * frame_bytes;
}

constexpr int kSquintThreads = 256;
constexpr int kSquintLdsBytes = 16384;

__global__ __launch_bounds__(kSquintThreads) void k_squint(
    const uint8_t* __restrict__ src0, const uint8_t* __restrict__ src1, const int* __restrict__ idx,
    const uint8_t* const* __restrict__ row_ptrs, int nsplit, int H, int W, int C, int k, int side, int ry, int vec16,
    SqDst dst) {
  __shared__ __attribute__((aligned(16))) uint8_t tile[kSquintLdsBytes];
  const int img = blockIdx.y;
  const int y0 = blockIdx.x * ry;
  const long long frame_bytes = (long long)H * W * C;
  const long long chunk_off = (long long)y0 * k * W * C;
  const int chunk_bytes = ry * k * W * C;
  const uint8_t* g = source_row(src0, src1, idx, row_ptrs, nsplit, img, frame_bytes) + chunk_off;
  if (vec16) {
    const uint4* g4 = reinterpret_cast<const uint4*>(g);
    uint4* t4 = reinterpret_cast<uint4*>(tile);
    for (int i = threadIdx.x; i < chunk_bytes / 16; i += kSquintThreads) t4[i] = g4[i];
  } else {
    for (int i = threadIdx.x; i < chunk_bytes; i += kSquintThreads) tile[i] = g[i];
  }
  if (dst.mode == kSqU8 && blockIdx.x == 0 && img < nsplit) ring_fields(dst, img);
  __syncthreads();
  const int n_out = C * ry * side;
  const float scale = (float)(255 * k * k);
  for (int o = threadIdx.x; o < n_out; o += kSquintThreads) {
    const int x = o % side;
    const int yl = (o / side) % ry;
    const int c = o / (side * ry);
    int s = 0;
    for (int i = 0; i < k; ++i) {
      const uint8_t* p = tile + ((yl * k + i) * W + x * k) * C + c;
      for (int j = 0; j < k; ++j) s += p[j * C];
    }
    emit(dst, img, nsplit, C, side, c, y0 + yl, x, s, k * k, scale);
  }
}

// Specialised path for a compile-time (channels C, factor K): a workgroup owns
// ry output rows (all 16 columns) of one image; thread t owns output pixel
// (t / 16, t % 16) for every channel.  The source rows are copied to LDS with
// batched 16-byte loads; each thread then reads its K x (K*C)-byte block rows as
// 32-bit words (K*C % 4 == 0) and adds each byte into its channel's sum, with
// every index known at compile time.
typedef unsigned u4v __attribute__((ext_vector_type(4)));   // 16-byte load / store unit

constexpr int kSquintCkLds = 40960;                 // LDS bytes of one k_squint_ck workgroup, at most
constexpr int kSquintCkMax16 = kSquintCkLds / 16;   // its 16-byte loads (a multiple of 256)

// lead > 0: the launch also draws the minibatch -- the first lead rows of
// workgroups (blockIdx.x == 0; dispatched first, so their latency-bound draws
// overlap the frame loads) take the draw's items, and the image workgroups
// compute their replay rows with the same Philox draw instead of reading idx
template <int C, int K, int SIDE>
__global__ __launch_bounds__(256) void k_squint_ck(const uint8_t* __restrict__ src0,
                                                   const uint8_t* __restrict__ src1, const int* __restrict__ idx,
                                                   const uint8_t* const* __restrict__ row_ptrs, int nsplit, int W,
                                                   int ry, SqDst dst, SampleArgs sa, int lead) {
  static_assert(256 % SIDE == 0, "whole output rows per workgroup");
  constexpr int SEG = K * C;          // bytes of one block row
  static_assert(SEG % 4 == 0, "32-bit block rows");
  extern __shared__ __attribute__((aligned(16))) uint8_t tile[];
  if ((int)blockIdx.y < lead) {
    const long long t = (long long)blockIdx.y * 256 + threadIdx.x;
    if (blockIdx.x == 0 && t < sample_items(sa.B, sa.A, sa.S)) sample_item(sa, t);
    return;
  }
  const int img = blockIdx.y - lead;
  const int y0 = blockIdx.x * ry;
  const int row_bytes = W * C;            // one source pixel row
  const long long frame_bytes = (long long)row_bytes * W;
  const int chunk16 = ry * K * row_bytes / 16;
  const uint8_t* frame =
      lead > 0 ? (img < nsplit ? src0 : src1) + (long long)sample_row(sa, img < nsplit ? img : img - nsplit) *
                                                 frame_bytes
               : source_row(src0, src1, idx, row_ptrs, nsplit, img, frame_bytes);
  const u4v* g4 = reinterpret_cast<const u4v*>(frame + (long long)y0 * K * row_bytes);
  u4v* t4 = reinterpret_cast<u4v*>(tile);
  // every load of the chunk is in flight before the first LDS store
  u4v v[kSquintCkMax16 / 256];
#pragma unroll
  for (int j = 0; j < kSquintCkMax16 / 256; ++j) {
    const int i = threadIdx.x + 256 * j;
    if (i < chunk16) v[j] = g4[i];
  }
  // a ring insertion's small fields move while the frame loads are in flight
  if (dst.mode == kSqU8 && blockIdx.x == 0 && img < nsplit) ring_fields(dst, img);
#pragma unroll
  for (int j = 0; j < kSquintCkMax16 / 256; ++j) {
    const int i = threadIdx.x + 256 * j;
    if (i < chunk16) t4[i] = v[j];
  }
  __syncthreads();
  const int yl = threadIdx.x / SIDE, x = threadIdx.x % SIDE;
  if (yl >= ry) return;
  int sum[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sum[c] = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const unsigned* w = reinterpret_cast<const unsigned*>(tile + (yl * K + r) * row_bytes + x * SEG);
#pragma unroll
    for (int q = 0; q < SEG / 4; ++q) {
      const unsigned v = w[q];
#pragma unroll
      for (int b = 0; b < 4; ++b) sum[(4 * q + b) % C] += (int)((v >> (8 * b)) & 0xFFu);
    }
  }
  const float scale = (float)(255 * K * K);
#pragma unroll
  for (int c = 0; c < C; ++c) emit(dst, img, nsplit, C, SIDE, c, y0 + yl, x, sum[c], K * K, scale);
}

// Frames already squinted at insertion (uint8 block means, [16, 16, C]): the
// k = 1 squint, x = q / 255 - 0.5.  One workgroup per image stages its bytes in
// LDS with 16-byte loads; thread p then emits pixel p of every channel (CHW
// stores, consecutive threads on consecutive pixels).
template <int C>
__global__ __launch_bounds__(256) void k_stored_ck(const uint8_t* __restrict__ src0,
                                                   const uint8_t* __restrict__ src1, const int* __restrict__ idx,
                                                   int nsplit, SqDst dst) {
  constexpr int SIDE = 16, BYTES = SIDE * SIDE * C;
  static_assert(BYTES % 16 == 0, "16-byte staging");
  __shared__ __attribute__((aligned(16))) uint8_t tile[BYTES];
  const int img = blockIdx.x;
  const uint4* g4 = reinterpret_cast<const uint4*>(source_row(src0, src1, idx, nullptr, nsplit, img, BYTES));
  if (threadIdx.x < BYTES / 16) reinterpret_cast<uint4*>(tile)[threadIdx.x] = g4[threadIdx.x];
  __syncthreads();
  const int p = threadIdx.x, y = p / SIDE, x = p % SIDE;
#pragma unroll
  for (int c = 0; c < C; ++c) emit(dst, img, nsplit, C, SIDE, c, y, x, tile[p * C + c], 1, 255.0f);
}

template <int C>
static bool try_stored(const uint8_t* s0, const uint8_t* s1, const int* idx, const uint8_t* const* rows, int nsplit,
                       int n, int H, int W, int Cr, int k, const SqDst& dst, hipStream_t st) {
  if (rows != nullptr || Cr != C || k != 1 || H != 16 || W != 16 || dst.mode == kSqU8) return false;
  if (dst.row_stride != (long long)C * 256 || (uintptr_t)s0 % 16 != 0 || (s1 && (uintptr_t)s1 % 16 != 0))
    return false;
  k_stored_ck<C><<<n, 256, 0, st>>>(s0, s1, idx, nsplit, dst);
  return true;
}

template <int C, int K, int SIDE>
static bool try_ck(const uint8_t* s0, const uint8_t* s1, const int* idx, const uint8_t* const* rows, int nsplit,
                   int n, int H, int W, int Cr, int kr, const SqDst& dst, hipStream_t st,
                   const SampleArgs* sa = nullptr) {
  if (Cr != C || kr != K || H != SIDE * K || W != H) return false;
  if (dst.mode != kSqU8 && dst.row_stride != (long long)C * SIDE * SIDE) return false;
  const long long frame_bytes = (long long)H * W * C;
  if (frame_bytes % 16 != 0 || (uintptr_t)s0 % 16 != 0 || (s1 && (uintptr_t)s1 % 16 != 0)) return false;
  const int row_bytes = K * W * C;
  int ry = 256 / SIDE < SIDE ? 256 / SIDE : SIDE;   // output rows of one workgroup: one thread per pixel
  while (ry > 1 && ry * row_bytes > kSquintCkLds) ry /= 2;
  if (ry * row_bytes > kSquintCkLds) return false;
  if ((ry * row_bytes) % 16 != 0) return false;
  const SampleArgs none{};
  const long long extra = sa ? (sample_items(sa->B, sa->A, sa->S) + 255) / 256 : 0;
  if (n + extra > 65535) return false;   // grid y limit
  dim3 grid(SIDE / ry, n + extra);
  k_squint_ck<C, K, SIDE><<<grid, 256, ry * row_bytes, st>>>(s0, s1, idx, rows, nsplit, W, ry, dst, sa ? *sa : none,
                                                             (int)extra);
  return true;
}

static int squint_rows_per_chunk(int W, int C, int k, int side) {
  const int row_bytes = k * W * C;
  int ry = side;
  // halve (keeping ry a divisor of side) while the chunk exceeds the LDS tile or
  // while halves would still carry >= 2 KB each: many small workgroups keep
  // enough loads in flight
  while (ry % 2 == 0 && (ry * row_bytes > kSquintLdsBytes || (ry / 2) * row_bytes >= 2048)) ry /= 2;
  if (ry * row_bytes > kSquintLdsBytes) ry = 1;
  return ry;
}

int squint_ok(int H, int W, int C, int k) {
  const int side = H / k;
  return (k * W * C) <= kSquintLdsBytes && side * k == H && (W / k) == side && side <= 64;
}

static int launch(const uint8_t* s0, const uint8_t* s1, const int* idx, const uint8_t* const* rows, int nsplit,
                  int n, int H, int W, int C, int k, const SqDst& dst, hipStream_t st) {
  // per-row pointers (serving) are only known on the device and may be unaligned:
  // they take the generic byte path
  if (rows == nullptr && (try_ck<9, 4, 16>(s0, s1, idx, rows, nsplit, n, H, W, C, k, dst, st) ||
                          try_ck<9, 8, 16>(s0, s1, idx, rows, nsplit, n, H, W, C, k, dst, st) ||
                          try_ck<3, 4, 16>(s0, s1, idx, rows, nsplit, n, H, W, C, k, dst, st) ||
                          try_ck<9, 4, 32>(s0, s1, idx, rows, nsplit, n, H, W, C, k, dst, st)))
    return launch_status("squint_ck");
  if (try_stored<9>(s0, s1, idx, rows, nsplit, n, H, W, C, k, dst, st) ||
      try_stored<3>(s0, s1, idx, rows, nsplit, n, H, W, C, k, dst, st))
    return launch_status("squint_stored");
  const int side = H / k;
  const int ry = squint_rows_per_chunk(W, C, k, side);
  const long long chunk_bytes = (long long)ry * k * W * C;
  const long long frame_bytes = (long long)H * W * C;
  const int vec16 = rows == nullptr && (chunk_bytes % 16 == 0) && (frame_bytes % 16 == 0) &&
                    ((uintptr_t)s0 % 16 == 0) && (s1 == nullptr || (uintptr_t)s1 % 16 == 0);
  dim3 grid(side / ry, n);
  k_squint<<<grid, kSquintThreads, 0, st>>>(s0, s1, idx, rows, nsplit, H, W, C, k, side, ry, vec16, dst);
  return launch_status("squint");
}

int launch_squint(const uint8_t* frames, const int* idx, int n, int H, int W, int C, int k, int bf16_out,
                  void* out, long long out_row_stride, hipStream_t st) {
  if (n == 0) return SQ_OK;
  const SqDst dst{bf16_out ? kSqBF16 : kSqF32, out, nullptr, out_row_stride, 0, 1, {}};
  return launch(frames, nullptr, idx, nullptr, n, n, H, W, C, k, dst, st);
}

int launch_squint_pair(const uint8_t* obs, const uint8_t* next_obs, const int* idx, int B, int H, int W, int C,
                       int k, float* out, hipStream_t st) {
  const int side = H / k;
  const SqDst dst{kSqF32, out, nullptr, (long long)C * side * side, 0, 1, {}};
  return launch(obs, next_obs, idx, nullptr, B, 2 * B, H, W, C, k, dst, st);
}

int launch_sample_squint(const SampleArgs& s, const uint8_t* obs, const uint8_t* next_obs, int H, int W, int C,
                         int k, float* out, hipStream_t st) {
  const int side = H / k, B = s.B;
  const SqDst dst{kSqF32, out, nullptr, (long long)C * side * side, 0, 1, {}};
  if (B > 0 && (try_ck<9, 4, 16>(obs, next_obs, nullptr, nullptr, B, 2 * B, H, W, C, k, dst, st, &s) ||
                try_ck<9, 8, 16>(obs, next_obs, nullptr, nullptr, B, 2 * B, H, W, C, k, dst, st, &s) ||
                try_ck<3, 4, 16>(obs, next_obs, nullptr, nullptr, B, 2 * B, H, W, C, k, dst, st, &s) ||
                try_ck<9, 4, 32>(obs, next_obs, nullptr, nullptr, B, 2 * B, H, W, C, k, dst, st, &s)))
    return launch_status("sample_squint");
  SQ_TRY(launch_sample_batch(s, st));
  return launch_squint_pair(obs, next_obs, s.idx, B, H, W, C, k, out, st);
}

int launch_squint_rows(const uint8_t* const* rows, int n, int H, int W, int C, int k, float* out, hipStream_t st) {
  if (n == 0) return SQ_OK;
  const int side = H / k;
  const SqDst dst{kSqF32, out, nullptr, (long long)C * side * side, 0, 1, {}};
  return launch(nullptr, nullptr, nullptr, rows, n, n, H, W, C, k, dst, st);
}

int launch_squint_insert(const uint8_t* obs, const uint8_t* next_obs, int n, int H, int W, int C, int k,
                         uint8_t* ring_obs, uint8_t* ring_next, int pos, int cap, const RingRows& f,
                         hipStream_t st) {
  if (n == 0) return SQ_OK;
  const SqDst dst{kSqU8, ring_obs, ring_next, 0, pos, cap, f};
  return launch(obs, next_obs, nullptr, nullptr, n, 2 * n, H, W, C, k, dst, st);
}

}  // namespace sq
