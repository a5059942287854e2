// Row-wise and small reduction kernels of the update, one wavefront (64 lanes)
// per row with cross-lane (DPP) reductions:
//   LayerNorm + activation forward / backward (Sec. IV Normalization)
//   column sums of gradient partials (bias, LayerNorm gain / shift gradients)
//   tanh-Gaussian policy head forward / backward (Sec. III Eq. (3))
//   twin-target softmax average + C51 projection (Eq. (1), categorical form)
//   cross entropy to the projected target, expected Q and its gradient
//   temperature step, per-update statistics and counters
// Every reduction has a fixed order: the DPP tree of wave_sum, and partial sums
// written per (row block, wave) and summed in order.
#include <math.h>

#include <type_traits>

#include "../common.h"
#include "bf16.h"
#include "tgauss.h"
#include "finish.h"

namespace sq {

constexpr int kLnRowsPerBlock = 8; // rows per workgroup (one per wave) in row-partial kernels

typedef float f4v __attribute__((ext_vector_type(4)));

// Cross-lane moves inside 16-lane rows (DPP): quad_perm [1,0,3,2] and [2,3,0,1],
// row_half_mirror, row_mirror.  Each step pairs lane i with a lane of the other
// half of its current group, so after the four steps every lane of a row holds
// the row's combined value (a + b and b + a round alike, so all lanes agree);
// the four row values are then read from lanes 0, 16, 32, 48 and combined as
// (r0 + r1) + (r2 + r3).  No LDS traffic, fixed order, result in every lane.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_read(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_move<0xB1>(v));
  v = fmaxf(v, dpp_move<0x4E>(v));
  v = fmaxf(v, dpp_move<0x141>(v));
  v = fmaxf(v, dpp_move<0x140>(v));
  return fmaxf(fmaxf(lane_read(v, 0), lane_read(v, 16)), fmaxf(lane_read(v, 32), lane_read(v, 48)));
}

// fixed-order block sum of 256 threads; result valid in every thread
__device__ float block_sum256(float v, float* sh) {
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

// ---------------------------------------------------------------- LayerNorm forward
// Lane j-mapping of a row of H floats: VEC (H a multiple of 256, 16-byte aligned
// rows): element t of the lane is column 256 (t / 4) + 4 lane + t % 4, read and
// written as float4; otherwise column lane + 64 t.  E = elements per lane.
template <int E, bool VEC>
__device__ __forceinline__ int ln_col(int lane, int t) {
  return VEC ? 256 * (t >> 2) + 4 * lane + (t & 3) : lane + 64 * t;
}

template <int E, bool VEC>
__device__ __forceinline__ void ln_load_row(const float* __restrict__ p, int H, int lane, float (&v)[E]) {
  if constexpr (VEC) {
#pragma unroll
    for (int c = 0; c < E / 4; ++c) {
      const f4v x = *reinterpret_cast<const f4v*>(__builtin_assume_aligned(p + 256 * c + 4 * lane, 16));
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 * c + e] = x[e];
    }
  } else {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int j = lane + 64 * t;
      v[t] = j < H ? p[j] : 0.f;
    }
  }
}

// a per-column parameter row (gain, shift) in the lane mapping above, read element by
// element (its start need not be 16-byte aligned); under VEC every column is < H
template <int E, bool VEC>
__device__ __forceinline__ void ln_load_par(const float* __restrict__ p, int H, int lane, float (&v)[E]) {
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int j = ln_col<E, VEC>(lane, t);
    if constexpr (VEC) v[t] = p[j];
    else v[t] = j < H ? p[j] : 0.f;
  }
}

template <int E, bool VEC>
__device__ __forceinline__ void ln_store_row(float* __restrict__ p, int H, int lane, const float (&v)[E]) {
  if constexpr (VEC) {
#pragma unroll
    for (int c = 0; c < E / 4; ++c)
      *reinterpret_cast<f4v*>(__builtin_assume_aligned(p + 256 * c + 4 * lane, 16)) =
          f4v{v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]};
  } else {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int j = lane + 64 * t;
      if (j < H) p[j] = v[t];
    }
  }
}

// the same row's bfloat16 copy (8-byte stores in the VEC mapping)
template <int E, bool VEC>
__device__ __forceinline__ void ln_store_row_h(uint16_t* __restrict__ p, int H, int lane, const float (&v)[E]) {
  if constexpr (VEC) {
#pragma unroll
    for (int c = 0; c < E / 4; ++c) {
      typedef unsigned u2v __attribute__((ext_vector_type(2)));
      const u2v w{(unsigned)bf16_bits(v[4 * c]) | ((unsigned)bf16_bits(v[4 * c + 1]) << 16),
                  (unsigned)bf16_bits(v[4 * c + 2]) | ((unsigned)bf16_bits(v[4 * c + 3]) << 16)};
      *reinterpret_cast<u2v*>(__builtin_assume_aligned(p + 256 * c + 4 * lane, 8)) = w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int j = lane + 64 * t;
      if (j < H) p[j] = bf16_bits(v[t]);
    }
  }
}

// one row per wave; the row, gain and shift are all requested before the reductions;
// yh (nullable): the bfloat16 copy of y, written alongside
template <int E, bool VEC>
__device__ __forceinline__ void ln_fwd_row(const float* __restrict__ pre, long long ld_pre, long long sz_pre,
                                           int rows, int H, const float* __restrict__ g,
                                           const float* __restrict__ beta, long long sz_par, int act_tanh,
                                           float* __restrict__ y, long long ld_y, long long sz_y,
                                           uint16_t* __restrict__ yh, int y32,
                                           float* __restrict__ xhat, float* __restrict__ rstd,
                                           const float* __restrict__ e1, long long ld_e1, int w1,
                                           const float* __restrict__ e2, long long ld_e2, int w2,
                                           const LnGroups& grp, int row, int z, int lane) {
  const bool second = z >= grp.zalt;
  const float* gz = second ? grp.g_alt + (z - grp.zalt) * sz_par : g + z * sz_par;
  const float* bz = second ? grp.beta_alt + (z - grp.zalt) * sz_par : beta + z * sz_par;
  float v[E], gv[E], bv[E];
  ln_load_row<E, VEC>(pre + z * sz_pre + row * ld_pre, H, lane, v);
  ln_load_par<E, VEC>(gz, H, lane, gv);
  ln_load_par<E, VEC>(bz, H, lane, bv);
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < E; ++t) s += v[t];
  const float mean = wave_sum(s) / (float)H;
  float q = 0.f;
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const float dv = ln_col<E, VEC>(lane, t) < H ? v[t] - mean : 0.f;
    q += dv * dv;
  }
  const float var = wave_sum(q) / (float)H;
  const float rs = 1.0f / sqrtf(var + 1e-5f);
  float xh[E], o[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    xh[t] = (v[t] - mean) * rs;
    const float a = __builtin_fmaf(gv[t], xh[t], bv[t]);   // the backward recomputes it bit for bit
    o[t] = act_tanh ? tanhf(a) : fmaxf(a, 0.f);
  }
  float* yr = y + z * sz_y + row * ld_y;
  uint16_t* yhr = yh ? yh + z * sz_y + row * ld_y : nullptr;
  const bool save = !second || grp.save_alt;
  if (save) ln_store_row<E, VEC>(xhat + ((long long)z * rows + row) * H, H, lane, xh);
  if (y32) ln_store_row<E, VEC>(yr, H, lane, o);
  if (yhr) ln_store_row_h<E, VEC>(yhr, H, lane, o);
  if (save && lane == 0) rstd[(long long)z * rows + row] = rs;
  const float* e1z = e1 + z * grp.sz_e1;
  const float* e2z = second && grp.e2_alt ? grp.e2_alt : e2;
  for (int j = lane; j < w1; j += 64) {
    const float t = e1z[row * ld_e1 + j];
    yr[H + j] = t;
    if (yhr) yhr[H + j] = bf16_bits(t);
  }
  for (int j = lane; j < w2; j += 64) {
    const float t = e2z[row * ld_e2 + j];
    yr[H + w1 + j] = t;
    if (yhr) yhr[H + w1 + j] = bf16_bits(t);
  }
}

// rows (one per wave) per LayerNorm forward workgroup: 8 measured 0.2-0.5 % more
// bfloat16 updates/s than 4 (half the workgroups, the same per-row work)
constexpr int kLnFwdRows = 8;

template <int E, bool VEC>
__global__ __launch_bounds__(64 * kLnFwdRows) void k_ln_fwd(const float* __restrict__ pre, long long ld_pre, long long sz_pre,
                                                int rows, int H, const float* __restrict__ g,
                                                const float* __restrict__ beta, long long sz_par, int act_tanh,
                                                float* __restrict__ y, long long ld_y, long long sz_y,
                                                uint16_t* __restrict__ yh, int y32,
                                                float* __restrict__ xhat, float* __restrict__ rstd,
                                                const float* __restrict__ e1, long long ld_e1, int w1,
                                                const float* __restrict__ e2, long long ld_e2, int w2,
                                                LnGroups grp) {
  const int row = blockIdx.x * kLnFwdRows + (threadIdx.x >> 6);
  if (row >= rows) return;
  ln_fwd_row<E, VEC>(pre, ld_pre, sz_pre, rows, H, g, beta, sz_par, act_tanh, y, ld_y, sz_y, yh, y32, xhat, rstd,
                     e1, ld_e1, w1, e2, ld_e2, w2, grp, row, blockIdx.y, threadIdx.x & 63);
}

// row-block b (kLnFwdRows rows) of a job: batch b / cdiv(rows, kLnFwdRows)
template <int E, bool VEC>
__device__ __forceinline__ void ln_fwd_job_block(const LnFwdJob& j, int b) {
  const int rb = (j.rows + kLnFwdRows - 1) / kLnFwdRows;
  const int row = (b % rb) * kLnFwdRows + (threadIdx.x >> 6);
  if (row >= j.rows) return;
  ln_fwd_row<E, VEC>(j.pre, j.ld_pre, j.sz_pre, j.rows, j.H, j.g, j.beta, j.sz_par, j.act_tanh, j.y, j.ld_y, j.sz_y,
                     j.yh, j.y32, j.xhat, j.rstd, j.e1, j.ld_e1, j.w1, j.e2, j.ld_e2, j.w2, j.grp, row, b / rb,
                     threadIdx.x & 63);
}

// two LayerNorm problems of the same width in one launch: workgroups [0, blocks0)
// take j0, the rest j1
template <int E, bool VEC>
__global__ __launch_bounds__(64 * kLnFwdRows) void k_ln_fwd_pair(LnFwdJob j0, LnFwdJob j1, int blocks0) {
  const int b = blockIdx.x;
  if (b < blocks0) ln_fwd_job_block<E, VEC>(j0, b);
  else ln_fwd_job_block<E, VEC>(j1, b - blocks0);
}

static bool al16(const void* p, long long a = 0, long long b = 0) {
  return (uintptr_t)p % 16 == 0 && a % 4 == 0 && b % 4 == 0;
}

// E = elements per lane (a power of two covering H), VEC as above
template <class F>
static int ln_dispatch(int H, bool vec_ok, F&& f) {
  if (vec_ok && H == 256) return f(std::integral_constant<int, 4>{}, std::true_type{});
  if (vec_ok && H == 512) return f(std::integral_constant<int, 8>{}, std::true_type{});
  if (vec_ok && H == 1024) return f(std::integral_constant<int, 16>{}, std::true_type{});
  if (H <= 64) return f(std::integral_constant<int, 1>{}, std::false_type{});
  if (H <= 128) return f(std::integral_constant<int, 2>{}, std::false_type{});
  if (H <= 256) return f(std::integral_constant<int, 4>{}, std::false_type{});
  if (H <= 512) return f(std::integral_constant<int, 8>{}, std::false_type{});
  return f(std::integral_constant<int, 16>{}, std::false_type{});
}

// whether the LayerNorm forward stores y in FP32: always, unless its owner dropped
// the FP32 values of y's buffer (a ReLU output with a bfloat16 copy, no copied
// columns: the backward recomputes the ReLU mask from x-hat, gain and shift)
static int ln_keeps_fp32(const float* y, const uint16_t* yh, int act_tanh, int extra_cols) {
  return (yh && !act_tanh && extra_cols == 0 && fp32_dropped(y)) ? 0 : 1;
}

// elements of y a LayerNorm forward writes, from its first
static long long ln_out_extent(int rows, int H, int batch, long long ld_y, long long sz_y, int w1, int w2) {
  if (rows <= 0 || batch <= 0) return 0;
  return (long long)(batch - 1) * sz_y + (long long)(rows - 1) * ld_y + H + w1 + w2;
}

int ln_act_fwd(const float* pre, long long ld_pre, long long sz_pre, int rows, int H, int batch, const float* g,
               const float* beta, long long sz_par, int act_tanh, float* y, long long ld_y, long long sz_y,
               float* xhat, float* rstd, const float* e1, long long ld_e1, int w1, const float* e2,
               long long ld_e2, int w2, hipStream_t st, const LnGroups* groups) {
  if (rows <= 0) return SQ_OK;
  const LnGroups grp = groups ? *groups : LnGroups{kNoAlt, nullptr, nullptr, 0, nullptr};
  const bool vec = al16(pre, ld_pre, sz_pre) && al16(y, ld_y, sz_y) && al16(xhat, H);
  uint16_t* yh = twin_of(y, ln_out_extent(rows, H, batch, ld_y, sz_y, w1, w2));
  const int y32 = ln_keeps_fp32(y, yh, act_tanh, w1 + w2);
  dim3 grid(cdiv(rows, kLnFwdRows), batch);
  return ln_dispatch(H, vec, [&](auto e, auto v) {
    k_ln_fwd<decltype(e)::value, decltype(v)::value><<<grid, 64 * kLnFwdRows, 0, st>>>(
        pre, ld_pre, sz_pre, rows, H, g, beta, sz_par, act_tanh, y, ld_y, sz_y, yh, y32, xhat, rstd, e1, ld_e1, w1,
        e2, ld_e2, w2, grp);
    return launch_status("ln_fwd");
  });
}

LnFwdJob ln_fwd_job(const float* pre, long long ld_pre, long long sz_pre, int rows, int H, int batch, const float* g,
                    const float* beta, long long sz_par, int act_tanh, float* y, long long ld_y, long long sz_y,
                    float* xhat, float* rstd, const float* e1, long long ld_e1, int w1, const float* e2,
                    long long ld_e2, int w2, const LnGroups* groups) {
  uint16_t* yh = twin_of(y, ln_out_extent(rows, H, batch, ld_y, sz_y, w1, w2));
  return LnFwdJob{pre, ld_pre, sz_pre, rows, H, batch, g, beta, sz_par, act_tanh, y, ld_y, sz_y, xhat, rstd, e1,
                  ld_e1, w1, e2, ld_e2, w2, groups ? *groups : LnGroups{kNoAlt, nullptr, nullptr, 0, nullptr},
                  yh, ln_keeps_fp32(y, yh, act_tanh, w1 + w2)};
}

static int ln_fwd_alone(const LnFwdJob& j, hipStream_t st) {
  return ln_act_fwd(j.pre, j.ld_pre, j.sz_pre, j.rows, j.H, j.batch, j.g, j.beta, j.sz_par, j.act_tanh, j.y, j.ld_y,
                    j.sz_y, j.xhat, j.rstd, j.e1, j.ld_e1, j.w1, j.e2, j.ld_e2, j.w2, st, &j.grp);
}

static bool ln_vec(const LnFwdJob& j) {
  return al16(j.pre, j.ld_pre, j.sz_pre) && al16(j.y, j.ld_y, j.sz_y) && al16(j.xhat, j.H);
}

int ln_act_fwd_pair(const LnFwdJob& j0, const LnFwdJob& j1, hipStream_t st) {
  if (j0.rows <= 0 || j1.rows <= 0 || j0.batch <= 0 || j1.batch <= 0 || j0.H != j1.H || ln_vec(j0) != ln_vec(j1)) {
    SQ_TRY(ln_fwd_alone(j0, st));
    return ln_fwd_alone(j1, st);
  }
  const int blocks0 = cdiv(j0.rows, kLnFwdRows) * j0.batch, blocks1 = cdiv(j1.rows, kLnFwdRows) * j1.batch;
  return ln_dispatch(j0.H, ln_vec(j0), [&](auto e, auto v) {
    k_ln_fwd_pair<decltype(e)::value, decltype(v)::value><<<blocks0 + blocks1, 64 * kLnFwdRows, 0, st>>>(j0, j1,
                                                                                                     blocks0);
    return launch_status("ln_fwd_pair");
  });
}

// ---------------------------------------------------------------- LayerNorm backward
// Per row: dz = dy * act'(y), dxh = dz * g,
//   dpre = rstd * (dxh - mean(dxh) - xhat * mean(dxh * xhat)).
// One row per wave, kLnRowsPerBlock rows (waves) per workgroup.  Column partials
// of the workgroup's rows, summed over its waves in order, go to
// part[z][3][blk][H] = (dpre, dz * xhat, dz) for the bias, gain and shift gradients.
template <int E, bool VEC>
__global__ __launch_bounds__(64 * kLnRowsPerBlock) void k_ln_bwd(
    const float* __restrict__ dy, long long ld_dy, long long sz_dy, const float* __restrict__ y, long long ld_y,
    long long sz_y, const float* __restrict__ xhat, const float* __restrict__ rstd, const float* __restrict__ g,
    const float* __restrict__ beta, long long sz_par, int rows, int H, int act_tanh, float* __restrict__ dpre,
    uint16_t* __restrict__ dpre_h, float* __restrict__ part) {
  extern __shared__ float shp[];   // [3][kLnRowsPerBlock][H] when partials are wanted
  constexpr int R = kLnRowsPerBlock;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = blockIdx.x, z = blockIdx.y;
  const int nblk = gridDim.x;
  const int row = blk * R + wave;
  const float* gz = g + z * sz_par;
  const float* bz = beta + z * sz_par;
  float pb[E], pg[E], pz[E];
#pragma unroll
  for (int t = 0; t < E; ++t) pb[t] = pg[t] = pz[t] = 0.f;
  if (row < rows) {
    // the activation's derivative: tanh' = 1 - y^2 from y; the ReLU mask from the
    // recomputed pre-activation fma(g, x-hat, shift) > 0 (y > 0 exactly when it is)
    // yv: y's row (tanh) or the shift (ReLU), one load pattern for both
    float dv[E], yv[E], xh[E], gv[E];
    ln_load_row<E, VEC>(dy + z * sz_dy + row * ld_dy, H, lane, dv);
    ln_load_row<E, VEC>(xhat + ((long long)z * rows + row) * H, H, lane, xh);
    ln_load_par<E, VEC>(gz, H, lane, gv);
    ln_load_par<E, VEC>(act_tanh ? y + z * sz_y + row * ld_y : bz, H, lane, yv);
    const float rs = rstd[(long long)z * rows + row];
    float dz[E];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const float yy = yv[t];
      dz[t] = dv[t] * (act_tanh ? (1.f - yy * yy) : (__builtin_fmaf(gv[t], xh[t], yy) > 0.f ? 1.f : 0.f));
      const float dx = dz[t] * gv[t];
      s1 += dx;
      s2 += dx * xh[t];
    }
    const float c1 = wave_sum(s1) / (float)H;
    const float c2 = wave_sum(s2) / (float)H;
#pragma unroll
    for (int t = 0; t < E; ++t) {
      pb[t] = rs * (dz[t] * gv[t] - c1 - xh[t] * c2);
      pg[t] = dz[t] * xh[t];
      pz[t] = dz[t];
    }
    ln_store_row<E, VEC>(dpre + ((long long)z * rows + row) * H, H, lane, pb);
    if (dpre_h) ln_store_row_h<E, VEC>(dpre_h + ((long long)z * rows + row) * H, H, lane, pb);
  }
  if (!part) return;
  ln_store_row<E, VEC>(shp + (0 * R + wave) * H, H, lane, pb);
  ln_store_row<E, VEC>(shp + (1 * R + wave) * H, H, lane, pg);
  ln_store_row<E, VEC>(shp + (2 * R + wave) * H, H, lane, pz);
  __syncthreads();
  float* pp = part + (long long)z * 3 * nblk * H + (long long)blk * H;
  for (int e = threadIdx.x; e < 3 * H; e += 64 * R) {
    const int k = e / H, j = e - k * H;
    const float* q = shp + k * R * H + j;
    float s = q[0];
#pragma unroll
    for (int w = 1; w < R; ++w) s += q[w * H];
    pp[(long long)k * nblk * H + j] = s;
  }
}

int ln_bwd_partial_rows(int rows) { return cdiv(rows, kLnRowsPerBlock); }

int ln_act_bwd(const float* dy, long long ld_dy, long long sz_dy, const float* y, long long ld_y, long long sz_y,
               const float* xhat, const float* rstd, const float* g, const float* beta, long long sz_par, int rows,
               int H, int batch, int act_tanh, float* dpre, float* partials, hipStream_t st) {
  if (rows <= 0) return SQ_OK;
  if (act_tanh ? !y : !beta) {
    set_error("ln_act_bwd: tanh needs y, ReLU needs the shift");
    return SQ_EINVAL;
  }
  dim3 grid(cdiv(rows, kLnRowsPerBlock), batch);
  const size_t lds = partials ? (size_t)3 * kLnRowsPerBlock * H * sizeof(float) : 0;
  const bool vec = al16(dy, ld_dy, sz_dy) && al16(xhat, H) && al16(dpre, H);
  uint16_t* dpre_h = twin_of(dpre, (long long)batch * rows * H);
  return ln_dispatch(H, vec, [&](auto e, auto v) {
    k_ln_bwd<decltype(e)::value, decltype(v)::value><<<grid, 64 * kLnRowsPerBlock, lds, st>>>(
        dy, ld_dy, sz_dy, y, ld_y, sz_y, xhat, rstd, g, beta, sz_par, rows, H, act_tanh, dpre, dpre_h, partials);
    return launch_status("ln_bwd");
  });
}

// ---------------------------------------------------------------- column partials
// Partial column sums of a [batch][rows][N] matrix over blocks of 4 rows:
// part[z][blk][N] (same blocking as the LayerNorm backward) -- used for the
// output-head bias gradients.
__global__ __launch_bounds__(256) void k_col_partials(const float* __restrict__ src, long long ld, long long sz,
                                                      int rows, int N, float* __restrict__ part) {
  const int blk = blockIdx.x, z = blockIdx.y, nblk = gridDim.x;
  for (int j = threadIdx.x; j < N; j += 256) {
    float s = 0.f;
    for (int rr = 0; rr < kLnRowsPerBlock; ++rr) {
      const int row = blk * kLnRowsPerBlock + rr;
      if (row < rows) s += src[z * sz + row * ld + j];
    }
    part[((long long)z * nblk + blk) * N + j] = s;
  }
}

int col_partials(const float* src, long long ld, long long sz, int rows, int N, int batch, float* part,
                 hipStream_t st) {
  if (rows <= 0) return SQ_OK;
  dim3 grid(cdiv(rows, kLnRowsPerBlock), batch);
  k_col_partials<<<grid, 256, 0, st>>>(src, ld, sz, rows, N, part);
  return launch_status("col_partials");
}

// Sum partial rows in order.  Segment s: part [batch][k][nrows][H] -> out[k][z * out_sz + c].
// A workgroup owns 64 columns of one (segment, z, k): wave w sums rows w, w+4, ...
// for its lane's column, then the four waves are added in order.
__global__ __launch_bounds__(256) void k_colsum(ColSegs segs) {
  __shared__ float sh[4][64];
  long long b = blockIdx.x;
  int s = 0;
  while (s < segs.n && b >= segs.s[s].count) { b -= segs.s[s].count; ++s; }
  if (s >= segs.n) return;
  const ColSeg& g = segs.s[s];
  const int cb = (g.H + 63) / 64;
  const int zk = (int)(b / cb);
  const int c0 = (int)(b - (long long)zk * cb) * 64;
  const int z = zk / g.k, kk = zk - z * g.k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = c0 + lane;
  float v = 0.f;
  if (c < g.H) {
    const float* p = g.part + ((long long)z * g.k + kk) * g.nrows * g.H + c;
    for (int r = wave; r < g.nrows; r += 4) v += p[(long long)r * g.H];
  }
  sh[wave][lane] = v;
  __syncthreads();
  if (wave == 0 && c < g.H && g.out[kk])
    g.out[kk][z * g.out_sz + c] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

int colsum(ColSegs segs, hipStream_t st) {
  long long total = 0;
  for (int i = 0; i < segs.n; ++i) {
    segs.s[i].count = (long long)segs.s[i].batch * segs.s[i].k * ((segs.s[i].H + 63) / 64);
    total += segs.s[i].count;
  }
  if (total == 0) return SQ_OK;
  k_colsum<<<(unsigned)total, 256, 0, st>>>(segs);
  return launch_status("colsum");
}

// ---------------------------------------------------------------- tanh-Gaussian head

// head [rows][2A] = [mu | u_s]; save [rows][3A] = (tanh u_s, sigma, action)
__global__ void k_tg_fwd(const float* __restrict__ head, int rows, int A, const float* __restrict__ eps, float lo,
                         float hi, float* __restrict__ action, float* __restrict__ logp, float* __restrict__ save) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const float* h = head + (long long)r * 2 * A;
  float lp = 0.f;
  for (int d = 0; d < A; ++d)
    lp += tanh_gauss_dim(h[d], h[A + d], eps[(long long)r * A + d], A, d, lo, hi, action + (long long)r * A,
                         save + (long long)r * 3 * A);
  if (logp) logp[r] = lp;
}

int tanh_gauss_fwd(const float* head, int rows, int A, const float* eps, float lo, float hi, float* action,
                   float* logp, float* save, hipStream_t st) {
  if (rows <= 0) return SQ_OK;
  k_tg_fwd<<<cdiv(rows, 64), 64, 0, st>>>(head, rows, A, eps, lo, hi, action, logp, save);
  return launch_status("tanh_gauss_fwd");
}

// d log pi / du = 2 tanh(u); d log pi / d log sigma = -1 (direct term).
// dlogp per row = (dlogp_vec ? dlogp_vec[r] : 0) + (dlogp_scalar ? *dlogp_scalar * scale : 0)
// One row per thread, kTgRows rows per workgroup; with part, the workgroup also
// writes the column sums of its rows of dhead (in row order) to part[blk][2A].
constexpr int kTgRows = 32;   // a partial row per 32 rows, as the GEMM epilogue's tiles
__global__ __launch_bounds__(kTgRows) void k_tg_bwd(const float* __restrict__ save, const float* __restrict__ eps,
                                                    const float* __restrict__ da, long long ld_da,
                                                    const float* __restrict__ dlogp_vec,
                                                    const float* __restrict__ dlogp_scalar, float scale, float lo,
                                                    float hi, int rows, int A, float* __restrict__ dhead,
                                                    int ldh, uint16_t* __restrict__ dhead_h,
                                                    float* __restrict__ part) {
  extern __shared__ float sht[];   // [kTgRows][2A] when part is wanted
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = r < rows;
  float dl = 0.f;
  if (live && dlogp_vec) dl += dlogp_vec[r];
  if (live && dlogp_scalar) dl += *dlogp_scalar * scale;
  for (int d = 0; d < A; ++d) {
    float du = 0.f, dls_out = 0.f;
    if (live) {
      const float tus = save[(long long)r * 3 * A + d];
      const float sd = save[(long long)r * 3 * A + A + d];
      const float a = save[(long long)r * 3 * A + 2 * A + d];
      const float e = eps[(long long)r * A + d];
      const float dav = da ? da[r * ld_da + d] : 0.f;
      du = dav * (1.f - a * a) + dl * 2.f * a;
      const float dls = du * sd * e - dl;
      dls_out = dls * 0.5f * (hi - lo) * (1.f - tus * tus);
      dhead[(long long)r * ldh + d] = du;
      dhead[(long long)r * ldh + A + d] = dls_out;
      if (dhead_h) {
        dhead_h[(long long)r * ldh + d] = bf16_bits(du);
        dhead_h[(long long)r * ldh + A + d] = bf16_bits(dls_out);
      }
    }
    if (part) {
      sht[threadIdx.x * 2 * A + d] = du;
      sht[threadIdx.x * 2 * A + A + d] = dls_out;
    }
  }
  if (!part) return;
  __syncthreads();
  for (int j = threadIdx.x; j < 2 * A; j += blockDim.x) {
    float sum = 0.f;
    for (int t = 0; t < (int)blockDim.x; ++t) sum += sht[t * 2 * A + j];
    part[(long long)blockIdx.x * 2 * A + j] = sum;
  }
}

int tanh_gauss_partial_rows(int rows) { return cdiv(rows, kTgRows); }

int tanh_gauss_bwd(const float* save, const float* eps, const float* da, long long ld_da, const float* dlogp_vec,
                   const float* dlogp_scalar, float scale, float lo, float hi, int rows, int A, float* dhead,
                   float* part, hipStream_t st, int ldh) {
  if (rows <= 0) return SQ_OK;
  if (ldh <= 0) ldh = 2 * A;
  const size_t lds = part ? (size_t)kTgRows * 2 * A * sizeof(float) : 0;
  uint16_t* dhead_h = twin_of(dhead, (long long)(rows - 1) * ldh + 2 * A);
  k_tg_bwd<<<cdiv(rows, kTgRows), kTgRows, lds, st>>>(save, eps, da, ld_da, dlogp_vec, dlogp_scalar, scale, lo, hi,
                                                     rows, A, dhead, ldh, dhead_h, part);
  return launch_status("tanh_gauss_bwd");
}

__global__ void k_mean_action(const float* __restrict__ head, int rows, int A, float* __restrict__ action) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * A) return;
  const int r = e / A, d = e - r * A;
  action[e] = tanhf(head[(long long)r * 2 * A + d]);
}

int mean_action(const float* head, int rows, int A, float* action, hipStream_t st) {
  if (rows <= 0) return SQ_OK;
  k_mean_action<<<cdiv((long long)rows * A, 256), 256, 0, st>>>(head, rows, A, action);
  return launch_status("mean_action");
}

// ---------------------------------------------------------------- C51 heads
constexpr int kMaxAtomsPerLane = 4;   // atoms up to 256

__device__ __forceinline__ void softmax_row(const float* l, int N, int lane, float* p) {
  float mx = -INFINITY;
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) {
    const int j = lane + 64 * t;
    if (j < N) mx = fmaxf(mx, l[j]);
  }
  mx = wave_max(mx);
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) {
    const int j = lane + 64 * t;
    p[t] = j < N ? expf(l[j] - mx) : 0.f;
    s += p[t];
  }
  s = wave_sum(s);
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) p[t] /= s;
}


// projection of one row, given the probabilities in registers (lane-strided:
// atom j lives in lane j % 64, slot j / 64).  Every lane walks all atoms j in
// order, reading p_j and b_j from their owner lane, so the sum order is fixed.
// Writes m and returns sum_i m_i z_i.
__device__ float project_row(const float* p, int N, int lane, float v_min, float dz, float r, float d, float gamma,
                             float bonus, float* m_out) {
  float bpos[kMaxAtomsPerLane];
  int nan_lane = 0;
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) {
    const int j = lane + 64 * t;
    const float zj = v_min + (float)j * dz;
    const float tz = r + gamma * (1.f - d) * (zj + bonus);
    const float q = (tz - v_min) / dz;
    nan_lane |= (j < N) & (q != q);
    bpos[t] = fminf(fmaxf(q, 0.f), (float)(N - 1));
  }
  // fminf / fmaxf drop a NaN; a row whose shifted atoms are not numbers gets a
  // NaN distribution instead (as the clamp of the definition keeps it)
  const bool nan_row = __any(nan_lane);
  float mi[kMaxAtomsPerLane];
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) mi[t] = 0.f;
#pragma unroll
  for (int ts = 0; ts < kMaxAtomsPerLane; ++ts) {
    if (64 * ts >= N) break;
    const int lim = N - 64 * ts < 64 ? N - 64 * ts : 64;
    for (int l = 0; l < lim; ++l) {
      const float pj = lane_read(p[ts], l);
      const float bj = lane_read(bpos[ts], l);
#pragma unroll
      for (int t = 0; t < kMaxAtomsPerLane; ++t)
        mi[t] += pj * fmaxf(0.f, 1.f - fabsf(bj - (float)(lane + 64 * t)));
    }
  }
  float mz = 0.f;
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) {
    const int i = lane + 64 * t;
    if (nan_row) mi[t] = __builtin_nanf("");
    if (i < N) {
      m_out[i] = mi[t];
      mz += mi[t] * (v_min + (float)i * dz);
    }
  }
  return wave_sum(mz);
}

// Projection of one row by segments.  The projected positions b_j are
// non-decreasing in j (every step from z_j to b_j is monotone, and so is its
// rounding), so their integer parts l_j are too, and the atoms j sharing an l form
// one contiguous segment.  Atom j's hat weight max(0, 1 - |b_j - i|) is 1 - f_j at
// i = l_j and f_j at l_j + 1 (f_j = b_j - l_j), zero elsewhere; so m_i is the sum of
// p (1 - f) over segment i plus the sum of p f over segment i - 1.  A segmented
// inclusive scan across the wave (fixed order, non-negative terms) leaves each
// segment's two sums at its last atom, which stores them at atoms l and l + 1 of
// the wave's LDS slices ma and mc; atoms that no segment reaches stay zero.  Every
// row costs the same, also one whose positions all coincide (a terminal
// transition puts every atom at the reward).
template <int T>
__device__ float project_row_t(const float (&p)[T], int N, int lane, float v_min, float dz, float r, float d,
                              float gamma, float bonus, float* ma, float* mc, float (&mi)[T]) {
  int nan_lane = 0;
  int l[T], hd[T];
  float a[T], c[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int j = lane + 64 * t;
    const float zj = v_min + (float)j * dz;
    const float tz = r + gamma * (1.f - d) * (zj + bonus);
    l[t] = N;          // past the last atom: a segment of its own, holding zeros
    a[t] = c[t] = 0.f;
    if (j < N) {
      const float q = (tz - v_min) / dz;
      nan_lane |= q != q;
      const float b = fminf(fmaxf(q, 0.f), (float)(N - 1));
      l[t] = (int)b;
      const float f = b - (float)l[t];
      a[t] = p[t] * (1.f - f);
      c[t] = p[t] * f;
      ma[j] = 0.f;
      mc[j] = 0.f;
    }
  }
  // fminf / fmaxf drop a NaN; a row whose shifted atoms are not numbers gets a
  // NaN distribution instead (as the clamp of the definition keeps it), so the
  // loss and the statistics of the update report it
  const bool nan_row = __any(nan_lane);
  // segment heads: the first atom, and every atom whose l differs from its predecessor's
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int prev = __shfl_up(l[t], 1);
    if (lane == 0) prev = t > 0 ? __builtin_amdgcn_readlane(l[t - 1], 63) : -1;
    hd[t] = l[t] != prev;
  }
  // scan each 64-atom slot; hd becomes "a head lies between the slot's start and here"
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float ya = __shfl_up(a[t], o), yc = __shfl_up(c[t], o);
      const int yh = __shfl_up(hd[t], o);
      if (lane >= o) {
        if (!hd[t]) {
          a[t] = ya + a[t];
          c[t] = yc + c[t];
        }
        hd[t] |= yh;
      }
    }
  }
  // atoms of a slot before its first head continue the previous slot's last segment
#pragma unroll
  for (int t = 1; t < T; ++t) {
    const float ca = lane_read(a[t - 1], 63), cc = lane_read(c[t - 1], 63);
    if (!hd[t]) {
      a[t] = ca + a[t];
      c[t] = cc + c[t];
    }
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the zeros land before the segment sums
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int j = lane + 64 * t;
    int next = __shfl_down(l[t], 1);
    if (lane == 63) next = t + 1 < T ? __builtin_amdgcn_readlane(l[t + 1], 0) : N;
    if (j < N && next != l[t]) {
      ma[l[t]] = a[t];
      if (l[t] + 1 < N) mc[l[t] + 1] = c[t];
    }
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  float mz = 0.f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int i = lane + 64 * t;
    float acc = i < N ? ma[i] + mc[i] : 0.f;
    if (nan_row) acc = __builtin_nanf("");
    mi[t] = acc;
    if (i < N) mz += acc * (v_min + (float)i * dz);
  }
  return wave_sum(mz);
}

// softmax of one row held lane-strided in registers (slots j >= N ignored)
template <int T>
__device__ __forceinline__ void softmax_regs(const float (&l)[T], int N, int lane, float (&p)[T]) {
  float mx = -INFINITY;
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (lane + 64 * t < N) mx = fmaxf(mx, l[t]);
  mx = wave_max(mx);
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    p[t] = lane + 64 * t < N ? expf(l[t] - mx) : 0.f;
    s += p[t];
  }
  s = wave_sum(s);
#pragma unroll
  for (int t = 0; t < T; ++t) p[t] /= s;
}

// logits4 [4][B][N]: online twins (0, 1) then target twins (2, 3).  Per row b:
// m = projection of the averaged target softmax (bonus -alpha log pi'), tgt_row = E_m[z];
// for each online twin: loss_row = CE(m, softmax), dlogits = (softmax - m) / B,
// q_row = E[z]; part (nullable): the workgroup's column sums of dlogits per twin.
// Every global input of a row is requested up front, so a wave waits on memory once.
template <int T, bool CDQ>
__global__ __launch_bounds__(64 * kLnRowsPerBlock) void k_target_ce(
    const float* __restrict__ logits4, int B, int N, float v_min, float v_max, const float* __restrict__ reward,
    const float* __restrict__ done, const float* __restrict__ logp_next, const float* __restrict__ log_alpha,
    float gamma, float* __restrict__ m_out, float* __restrict__ tgt_row, float* __restrict__ dlogits2, int ld_dl,
    uint16_t* __restrict__ dl_h, float* __restrict__ loss_row, float* __restrict__ q_row, float* __restrict__ part) {
  // [kLnRowsPerBlock][2][N] projected positions and probabilities of each wave's
  // row, then [2][kLnRowsPerBlock][N] head-bias partials when part is wanted
  extern __shared__ float shc2[];
  constexpr int R = kLnRowsPerBlock;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x * R + wave;
  float* shp = shc2 + 2 * R * N;
  const float dz = (v_max - v_min) / (float)(N - 1);
  const float invB = 1.0f / (float)B;
  float dl[2][T];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int t = 0; t < T; ++t) dl[i][t] = 0.f;
  if (b < B) {
    float lg[4][T];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int j = lane + 64 * t;
        lg[r][t] = j < N ? logits4[((long long)r * B + b) * N + j] : 0.f;
      }
    const float rb = reward[b], db = done[b], lpb = logp_next[b], la = *log_alpha;
    float p0[T], p1[T], mi[T];
    softmax_regs<T>(lg[2], N, lane, p0);
    softmax_regs<T>(lg[3], N, lane, p1);
    if constexpr (CDQ) {
      // clipped double-Q: the twin with the smaller expected value (twin 0 on ties)
      float e0 = 0.f, e1 = 0.f;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float zj = v_min + (float)(lane + 64 * t) * dz;
        e0 += p0[t] * zj;
        e1 += p1[t] * zj;
      }
      e0 = wave_sum(e0);
      e1 = wave_sum(e1);
      if (e1 < e0) {
#pragma unroll
        for (int t = 0; t < T; ++t) p0[t] = p1[t];
      }
    } else {
#pragma unroll
      for (int t = 0; t < T; ++t) p0[t] = 0.5f * (p0[t] + p1[t]);
    }
    const float mz = project_row_t<T>(p0, N, lane, v_min, dz, rb, db, gamma, -expf(la) * lpb, shc2 + 2 * wave * N,
                                      shc2 + (2 * wave + 1) * N, mi);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int j = lane + 64 * t;
      if (j < N) m_out[(long long)b * N + j] = mi[t];
    }
    if (lane == 0 && tgt_row) tgt_row[b] = mz;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      float mx = -INFINITY;
#pragma unroll
      for (int t = 0; t < T; ++t)
        if (lane + 64 * t < N) mx = fmaxf(mx, lg[i][t]);
      mx = wave_max(mx);
      float e[T], s = 0.f;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        e[t] = lane + 64 * t < N ? expf(lg[i][t] - mx) : 0.f;
        s += e[t];
      }
      s = wave_sum(s);
      const float lse = logf(s);
      float ce = 0.f, q = 0.f;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int j = lane + 64 * t;
        if (j < N) {
          const float pj = e[t] / s;
          ce -= mi[t] * (lg[i][t] - mx - lse);
          q += pj * (v_min + (float)j * dz);
          dl[i][t] = (pj - mi[t]) * invB;
          dlogits2[((long long)i * B + b) * ld_dl + j] = dl[i][t];
          if (dl_h) dl_h[((long long)i * B + b) * ld_dl + j] = bf16_bits(dl[i][t]);
        }
      }
      ce = wave_sum(ce);
      q = wave_sum(q);
      if (lane == 0) {
        loss_row[(long long)i * B + b] = ce;
        q_row[(long long)i * B + b] = q;
      }
    }
  }
  if (!part) return;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int j = lane + 64 * t;
      if (j < N) shp[(i * R + wave) * N + j] = dl[i][t];
    }
  __syncthreads();
  const int nblk = gridDim.x;
  for (int e = threadIdx.x; e < 2 * N; e += 64 * R) {
    const int i = e / N, j = e - i * N;
    float sum = shp[(i * R) * N + j];
    for (int w = 1; w < R; ++w) sum += shp[(i * R + w) * N + j];
    part[((long long)i * nblk + blockIdx.x) * N + j] = sum;
  }
}

template <bool CDQ>
static void launch_target_ce(const float* logits4, int B, int N, float v_min, float v_max, const float* reward,
                             const float* done, const float* logp_next, const float* log_alpha, float gamma, float* m,
                             float* tgt_row, float* dlogits2, int ld_dl, uint16_t* dl_h, float* loss_row,
                             float* q_row, float* part, hipStream_t st) {
  const size_t lds = (size_t)(part ? 4 : 2) * kLnRowsPerBlock * N * sizeof(float);
  const dim3 grid(cdiv(B, kLnRowsPerBlock)), block(64 * kLnRowsPerBlock);
  if (N <= 64)
    k_target_ce<1, CDQ><<<grid, block, lds, st>>>(logits4, B, N, v_min, v_max, reward, done, logp_next, log_alpha,
                                                  gamma, m, tgt_row, dlogits2, ld_dl, dl_h, loss_row, q_row, part);
  else if (N <= 128)
    k_target_ce<2, CDQ><<<grid, block, lds, st>>>(logits4, B, N, v_min, v_max, reward, done, logp_next, log_alpha,
                                                  gamma, m, tgt_row, dlogits2, ld_dl, dl_h, loss_row, q_row, part);
  else if (N <= 192)
    k_target_ce<3, CDQ><<<grid, block, lds, st>>>(logits4, B, N, v_min, v_max, reward, done, logp_next, log_alpha,
                                                  gamma, m, tgt_row, dlogits2, ld_dl, dl_h, loss_row, q_row, part);
  else
    k_target_ce<4, CDQ><<<grid, block, lds, st>>>(logits4, B, N, v_min, v_max, reward, done, logp_next, log_alpha,
                                                  gamma, m, tgt_row, dlogits2, ld_dl, dl_h, loss_row, q_row, part);
}

int target_ce(const float* logits4, int B, int N, float v_min, float v_max, const float* reward, const float* done,
              const float* logp_next, const float* log_alpha, float gamma, int cdq, float* m, float* tgt_row,
              float* dlogits2, float* loss_row, float* q_row, float* part, hipStream_t st, int ld_dl) {
  if (B <= 0) return SQ_OK;
  if (N < 2 || N > 64 * kMaxAtomsPerLane) return SQ_EINVAL;
  if (ld_dl <= 0) ld_dl = N;
  if (ld_dl < N) return SQ_EINVAL;
  uint16_t* dl_h = twin_of(dlogits2, (long long)(2 * B - 1) * ld_dl + N);
  if (cdq)
    launch_target_ce<true>(logits4, B, N, v_min, v_max, reward, done, logp_next, log_alpha, gamma, m, tgt_row,
                           dlogits2, ld_dl, dl_h, loss_row, q_row, part, st);
  else
    launch_target_ce<false>(logits4, B, N, v_min, v_max, reward, done, logp_next, log_alpha, gamma, m, tgt_row,
                            dlogits2, ld_dl, dl_h, loss_row, q_row, part, st);
  return launch_status("target_ce");
}

// Scalar critic (one output per twin; Eqs. (1)-(2)): per row,
// y = r + gamma (1 - d)(Qbar - alpha log pi'), Qbar the twin-target average or, with
// cdq, their minimum; each online twin's loss_row = (Q - y)^2, dlogits = 2 (Q - y) / B,
// q_row = Q; part (nullable): column sums of dlogits per block of
// kLnRowsPerBlock rows (thread order), one value per twin.
__global__ __launch_bounds__(64) void k_target_mse(const float* __restrict__ logits4, int B,
                                                   const float* __restrict__ reward, const float* __restrict__ done,
                                                   const float* __restrict__ logp_next,
                                                   const float* __restrict__ log_alpha, float gamma, int cdq,
                                                   float* __restrict__ tgt_row, float* __restrict__ dlogits2,
                                                   float* __restrict__ loss_row, float* __restrict__ q_row,
                                                   float* __restrict__ part) {
  constexpr int R = kLnRowsPerBlock;
  __shared__ float sh[2][R];
  const int t = threadIdx.x, b = blockIdx.x * R + t;
  if (t < R) {
    float dl[2] = {0.f, 0.f};
    if (b < B) {
      const float qa = logits4[(long long)2 * B + b], qb = logits4[(long long)3 * B + b];
      const float qn = cdq ? fminf(qa, qb) : 0.5f * (qa + qb);
      const float y = reward[b] + gamma * (1.f - done[b]) * (qn - expf(*log_alpha) * logp_next[b]);
      tgt_row[b] = y;
      for (int i = 0; i < 2; ++i) {
        const float q = logits4[(long long)i * B + b];
        const float diff = q - y;
        loss_row[(long long)i * B + b] = diff * diff;
        q_row[(long long)i * B + b] = q;
        dl[i] = 2.f * diff / (float)B;
        dlogits2[(long long)i * B + b] = dl[i];
      }
    }
    sh[0][t] = dl[0];
    sh[1][t] = dl[1];
  }
  __syncthreads();
  if (part && t < 2) {
    float s = sh[t][0];
    for (int w = 1; w < R; ++w) s += sh[t][w];
    part[(long long)t * gridDim.x + blockIdx.x] = s;
  }
}

int target_mse(const float* logits4, int B, const float* reward, const float* done, const float* logp_next,
               const float* log_alpha, float gamma, int cdq, float* tgt_row, float* dlogits2, float* loss_row,
               float* q_row, float* part, hipStream_t st) {
  if (B <= 0) return SQ_OK;
  k_target_mse<<<cdiv(B, kLnRowsPerBlock), 64, 0, st>>>(logits4, B, reward, done, logp_next, log_alpha, gamma, cdq,
                                                        tgt_row, dlogits2, loss_row, q_row, part);
  return launch_status("target_mse");
}

// plain projection of given probabilities (library entry point)
__global__ __launch_bounds__(256) void k_project(const float* __restrict__ p, const float* __restrict__ reward,
                                                 const uint8_t* __restrict__ done, const float* __restrict__ bonus,
                                                 float gamma, int B, int N, float v_min, float v_max,
                                                 float* __restrict__ m) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + wave;
  if (b >= B) return;
  float pr[kMaxAtomsPerLane];
#pragma unroll
  for (int t = 0; t < kMaxAtomsPerLane; ++t) {
    const int j = lane + 64 * t;
    pr[t] = j < N ? p[(long long)b * N + j] : 0.f;
  }
  const float dz = (v_max - v_min) / (float)(N - 1);
  project_row(pr, N, lane, v_min, dz, reward[b], done[b] ? 1.f : 0.f, gamma, bonus ? bonus[b] : 0.f,
              m + (long long)b * N);
}

int c51_project_raw(const float* p, const float* reward, const uint8_t* done, const float* bonus, float gamma, int B,
                    int N, float v_min, float v_max, float* m, hipStream_t st) {
  if (B <= 0) return SQ_OK;
  k_project<<<cdiv(B, 4), 256, 0, st>>>(p, reward, done, bonus, gamma, B, N, v_min, v_max, m);
  return launch_status("c51_project");
}

// actor-loss head: Q_i = sum_j p_ij z_j, dL/dl_ij = -(1 / (2B)) p_ij (z_j - Q_i),
// qa_row[b] = (Q_1 + Q_2) / 2
__global__ __launch_bounds__(256) void k_expq(const float* __restrict__ logits2, int B, int N, float v_min,
                                              float v_max, float* __restrict__ dlogits2, int ld_dl,
                                              uint16_t* __restrict__ dl_h, float* __restrict__ qa_row) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + wave;
  if (b >= B) return;
  const float dz = (v_max - v_min) / (float)(N - 1);
  const float c = -0.5f / (float)B;
  float qsum = 0.f;
  for (int i = 0; i < 2; ++i) {
    float p[kMaxAtomsPerLane];
    softmax_row(logits2 + ((long long)i * B + b) * N, N, lane, p);
    float q = 0.f;
#pragma unroll
    for (int t = 0; t < kMaxAtomsPerLane; ++t) {
      const int j = lane + 64 * t;
      if (j < N) q += p[t] * (v_min + (float)j * dz);
    }
    q = wave_sum(q);
#pragma unroll
    for (int t = 0; t < kMaxAtomsPerLane; ++t) {
      const int j = lane + 64 * t;
      if (j < N) {
        const float g = c * p[t] * ((v_min + (float)j * dz) - q);
        dlogits2[((long long)i * B + b) * ld_dl + j] = g;
        if (dl_h) dl_h[((long long)i * B + b) * ld_dl + j] = bf16_bits(g);
      }
    }
    qsum += q;
  }
  if (lane == 0) qa_row[b] = 0.5f * qsum;
}

int expected_q_grad(const float* logits2, int B, int N, float v_min, float v_max, float* dlogits2, float* qa_row,
                    hipStream_t st, int ld_dl) {
  if (B <= 0) return SQ_OK;
  if (ld_dl <= 0) ld_dl = N;
  if (ld_dl < N) return SQ_EINVAL;
  uint16_t* dl_h = twin_of(dlogits2, (long long)(2 * B - 1) * ld_dl + N);
  k_expq<<<cdiv(B, 4), 256, 0, st>>>(logits2, B, N, v_min, v_max, dlogits2, ld_dl, dl_h, qa_row);
  return launch_status("expected_q");
}

// ---------------------------------------------------------------- end of an update
// stats = {L_c, L_pi, L_alpha, alpha_new, entropy, mean Q, mean target, non-finite}
// actor-loss head of a scalar critic: qa_row[b] = (Q_1 + Q_2) / 2, dL/dQ_i = -1 / (2B)
__global__ __launch_bounds__(256) void k_expq_scalar(const float* __restrict__ q2, int B, float* __restrict__ dq2,
                                                     float* __restrict__ qa_row) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const float c = -0.5f / (float)B;
  dq2[b] = c;
  dq2[(long long)B + b] = c;
  qa_row[b] = 0.5f * (q2[b] + q2[(long long)B + b]);
}

int expected_q_scalar(const float* q2, int B, float* dq2, float* qa_row, hipStream_t st) {
  if (B <= 0) return SQ_OK;
  k_expq_scalar<<<cdiv(B, 256), 256, 0, st>>>(q2, B, dq2, qa_row);
  return launch_status("expected_q_scalar");
}

__global__ __launch_bounds__(256) void k_finish(FinishJob f) { finish_block(f); }

int finish_update(const float* loss_row, const float* q_row, const float* tgt_row, const float* logp,
                  const float* qa_row, const float* scal, int B, int actor_step, int* ctr, float* stats,
                  hipStream_t st) {
  k_finish<<<1, 256, 0, st>>>(FinishJob{loss_row, q_row, tgt_row, logp, qa_row, scal, B, actor_step, ctr, stats});
  return launch_status("finish_update");
}

// ---------------------------------------------------------------- conv bias gradient
// db[f] = sum over (n, p) of dout * (out > 0): workgroup (chunk, f) sums a fixed
// chunk of the (n, p) range into part[chunk][f]; colsum adds the chunks in order.
__global__ __launch_bounds__(256) void k_conv_bias(const float* __restrict__ dout, const float* __restrict__ out,
                                                   int n, int F, int HW, int per_chunk, float* __restrict__ part) {
  __shared__ float sh[256];
  const int f = blockIdx.y, ch = blockIdx.x;
  const long long total = (long long)n * HW;
  const long long e0 = (long long)ch * per_chunk;
  const long long e1 = e0 + per_chunk < total ? e0 + per_chunk : total;
  float s = 0.f;
  for (long long e = e0 + threadIdx.x; e < e1; e += 256) {
    const long long nn = e / HW, p = e - nn * HW;
    const long long i = (nn * F + f) * HW + p;
    s += out[i] > 0.f ? dout[i] : 0.f;
  }
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) part[(long long)ch * F + f] = s;
}

int conv_bias_chunks(int n, int HW) {
  const long long total = (long long)n * HW;
  int chunks = cdiv(total, 2048);
  return chunks < 1 ? 1 : (chunks > 256 ? 256 : chunks);
}

int conv_bias_grad(const float* dout, const float* out, int n, int F, int HW, float* db, float* part,
                   hipStream_t st) {
  if (n <= 0) return SQ_OK;
  const int chunks = conv_bias_chunks(n, HW);
  const int per = cdiv((long long)n * HW, chunks);
  k_conv_bias<<<dim3(chunks, F), 256, 0, st>>>(dout, out, n, F, HW, per, part);
  SQ_TRY(launch_status("conv_bias_grad"));
  ColSegs s{};
  s.n = 1;
  s.s[0] = ColSeg{part, chunks, F, 1, 1, {db, nullptr, nullptr}, 0, 0};
  return colsum(s, st);
}

}  // namespace sq
