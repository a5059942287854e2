// Fused conv encoder for 16x16 squinted images (Sec. IV Encoder Design Choices):
// 3x3 valid convolutions, the first with stride 2, ReLU after each.
//
// Forward: a workgroup owns G images.  The images and every intermediate
// activation stay in LDS; each convolution is an implicit GEMM on the matrix
// cores (rows = output pixels of the G images, columns = output channels,
// k = (input channel, ky, kx)) whose operand fragments are gathered straight
// from LDS (activations) and from the weight rows (L1/L2 resident).  Outputs of
// every layer are also written to HBM for the backward pass.
//
// Backward: the same workgroup shape.  Per layer, from the gradient at the
// layer's output: the ReLU mask, the weight-gradient contribution of the G
// images (contraction over their output pixels), the bias contribution, and the
// input gradient (a transposed convolution) for the layer below -- all in LDS.
// Each workgroup writes its partial encoder gradient; a second kernel adds the
// partials in workgroup order, so the result is deterministic.
#include "../common.h"
#include "bf16.h"

namespace sq {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kEncThreads = 256;

// 16x16 output tile += A(16 x K) B(K x 16); A(r, k) and B(k, c) are gathered by
// functors (zero outside the valid range).  Wave-level: every lane participates.
// The bfloat16 form rounds both operands to bfloat16 values and multiplies them
// on the FP32 matrix cores: a product of two bfloat16 values is exact in FP32
// and the accumulation is FP32, as on the bfloat16 units, while the gathers keep
// the register footprint (and occupancy) of the FP32 form.
template <bool BF16, class FA, class FB>
__device__ __forceinline__ v4f mma_tile(const FA& fa, const FB& fb, int K, v4f acc) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + lq;
    float a = k < K ? fa(li, k) : 0.f;
    float b = k < K ? fb(k, li) : 0.f;
    if constexpr (BF16) {
      a = bf16_round(a);
      b = bf16_round(b);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// geometry of layer l (0-based): input side, output side, stride
__host__ __device__ constexpr int enc_in(int l) { return l == 0 ? 16 : (l == 1 ? 7 : (l == 2 ? 5 : 3)); }
__host__ __device__ constexpr int enc_out(int l) { return l == 0 ? 7 : (l == 1 ? 5 : (l == 2 ? 3 : 1)); }
__host__ __device__ constexpr int enc_stride(int l) { return l == 0 ? 2 : 1; }

// ---------------------------------------------------------------- forward
// One conv layer of the gn (<= G) present images: in_lds [G][CIN][HI][HI] ->
// post-ReLU out_lds [G][F][HO][HO] (nullable) and out_g (NCHW rows of the images).
template <bool BF16, int G, int CIN, int F, int HI, int HO, int S>
__device__ void conv_layer_fwd(const float* in_lds, float* out_lds, const float* __restrict__ W,
                               const float* __restrict__ bias, float* __restrict__ out_g, int gn) {
  constexpr int P = HO * HO;            // output pixels per image
  constexpr int ROWS = G * P;
  constexpr int K = CIN * 9;
  constexpr int RT = (ROWS + 15) / 16, CT = F / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = wave; t < RT * CT; t += kEncThreads / 64) {
    const int rt = t / CT, ct = t - rt * CT;
    const int r0 = rt * 16, c0 = ct * 16;
    auto fa = [&](int r, int k) -> float {
      const int row = r0 + r;
      if (row >= ROWS) return 0.f;
      const int g = row / P, p = row - g * P, oy = p / HO, ox = p - oy * HO;
      const int c = k / 9, tt = k - 9 * c, ky = tt / 3, kx = tt - 3 * ky;
      return in_lds[((g * CIN + c) * HI + oy * S + ky) * HI + ox * S + kx];
    };
    auto fb = [&](int k, int c) -> float { return W[(c0 + c) * K + k]; };
    v4f acc = mma_tile<BF16>(fa, fb, K, v4f{0.f, 0.f, 0.f, 0.f});
    const int col = c0 + (lane & 15);
    const float bv = bias[col];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = r0 + 4 * (lane >> 4) + q;
      if (row < ROWS) {
        const int g = row / P, p = row - g * P;
        const float v = fmaxf(acc[q] + bv, 0.f);
        if (out_lds) out_lds[(g * F + col) * P + p] = v;
        if (g < gn) out_g[((long long)g * F + col) * P + p] = v;
      }
    }
  }
}

template <bool BF16, int G, int C, int F, int NC>
__global__ __launch_bounds__(kEncThreads) void k_encoder_fwd(const float* __restrict__ x, int n,
                                                             const float* __restrict__ W0, const float* __restrict__ b0,
                                                             const float* __restrict__ W1, const float* __restrict__ b1,
                                                             const float* __restrict__ W2, const float* __restrict__ b2,
                                                             float* __restrict__ h0, float* __restrict__ h1,
                                                             float* __restrict__ h2) {
  constexpr int X = G * C * 256, A0 = G * F * 49, A1 = G * F * 25;
  __shared__ float lx[X];
  __shared__ float la0[A0];
  __shared__ float la1[A1];
  const int img0 = blockIdx.x * G;
  const int gn = n - img0 < G ? n - img0 : G;
  // images of this group; the missing images of a ragged tail read as zeros
  for (int e = threadIdx.x; e < X; e += kEncThreads) {
    const int g = e / (C * 256);
    lx[e] = g < gn ? x[(long long)img0 * C * 256 + e] : 0.f;
  }
  __syncthreads();
  conv_layer_fwd<BF16, G, C, F, 16, 7, 2>(lx, la0, W0, b0, h0 + (long long)img0 * F * 49, gn);
  __syncthreads();
  conv_layer_fwd<BF16, G, F, F, 7, 5, 1>(la0, NC > 2 ? la1 : nullptr, W1, b1, h1 + (long long)img0 * F * 25, gn);
  if constexpr (NC > 2) {
    __syncthreads();
    conv_layer_fwd<BF16, G, F, F, 5, 3, 1>(la1, nullptr, W2, b2, h2 + (long long)img0 * F * 9, gn);
  }
}

// ---------------------------------------------------------------- backward
// Layer l of the G images, from dcur = gradient at its post-ReLU output:
//   dpre = dcur * (out > 0)                                   (in place)
//   part[W_off + f*K + k] = sum_{g,p} dpre[g][f][p] patch(in)[g][p][k]
//   part[b_off + f]       = sum_{g,p} dpre[g][f][p]
//   dprev[g][c][iy][ix]   = sum_{f,ky,kx} dpre[g][f][iy-ky][ix-kx] W[f][c][ky][kx]   (stride-1 layers, if wanted)
template <bool BF16, int G, int CIN, int F, int HI, int HO, int S, bool DX>
__device__ void conv_layer_bwd(float* dcur, const float* __restrict__ out_g, const float* in_lds,
                               const float* __restrict__ W, float* __restrict__ partW, float* __restrict__ partb,
                               float* dprev, int gn) {
  constexpr int P = HO * HO;
  constexpr int K = CIN * 9;
  constexpr int NPOS = G * P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // ReLU mask (tail images carry zero gradient)
  for (int e = threadIdx.x; e < G * F * P; e += kEncThreads) {
    const int g = e / (F * P);
    dcur[e] = (g < gn && out_g[e] > 0.f) ? dcur[e] : 0.f;
  }
  __syncthreads();
  // bias: thread f sums its channel over the G images in order
  if (threadIdx.x < F) {
    const int f = threadIdx.x;
    float sb = 0.f;
    for (int g = 0; g < G; ++g)
      for (int p = 0; p < P; ++p) sb += dcur[(g * F + f) * P + p];
    partb[f] = sb;
  }
  // weights: rows f (F/16 tiles), columns k (K padded to 16), contraction over positions
  {
    constexpr int RT = F / 16, CT = (K + 15) / 16;
    for (int t = wave; t < RT * CT; t += kEncThreads / 64) {
      const int rt = t / CT, ct = t - rt * CT;
      const int f0 = rt * 16, k0 = ct * 16;
      auto fa = [&](int r, int q) -> float {      // A(f, pos) = dpre
        const int g = q / P, p = q - g * P;
        return dcur[(g * F + f0 + r) * P + p];
      };
      auto fb = [&](int q, int c) -> float {      // B(pos, k) = patch
        const int k = k0 + c;
        if (k >= K) return 0.f;
        const int g = q / P, p = q - g * P, oy = p / HO, ox = p - oy * HO;
        const int ci = k / 9, tt = k - 9 * ci, ky = tt / 3, kx = tt - 3 * ky;
        return in_lds[((g * CIN + ci) * HI + oy * S + ky) * HI + ox * S + kx];
      };
      const v4f acc = mma_tile<BF16>(fa, fb, NPOS, v4f{0.f, 0.f, 0.f, 0.f});
      const int kk = k0 + (lane & 15);
      if (kk < K) {
#pragma unroll
        for (int q = 0; q < 4; ++q) partW[(f0 + 4 * (lane >> 4) + q) * K + kk] = acc[q];
      }
    }
  }
  if constexpr (DX) {
    static_assert(S == 1, "input gradients are needed for stride-1 layers only");
    // rows (g, iy, ix), columns c (CIN/16 tiles), contraction k = (f, ky, kx)
    constexpr int ROWS = G * HI * HI;
    constexpr int RT = (ROWS + 15) / 16, CT = CIN / 16, KT = F * 9;
    for (int t = wave; t < RT * CT; t += kEncThreads / 64) {
      const int rt = t / CT, ct = t - rt * CT;
      const int r0 = rt * 16, c0 = ct * 16;
      auto fa = [&](int r, int k) -> float {
        const int row = r0 + r;
        if (row >= ROWS) return 0.f;
        const int g = row / (HI * HI), q = row - g * HI * HI, iy = q / HI, ix = q - iy * HI;
        const int f = k / 9, tt = k - 9 * f, ky = tt / 3, kx = tt - 3 * ky;
        const int oy = iy - ky, ox = ix - kx;
        if (oy < 0 || oy >= HO || ox < 0 || ox >= HO) return 0.f;
        return dcur[(g * F + f) * P + oy * HO + ox];
      };
      auto fb = [&](int k, int c) -> float {
        const int f = k / 9, tt = k - 9 * f;
        return W[(f * CIN + c0 + c) * 9 + tt];
      };
      const v4f acc = mma_tile<BF16>(fa, fb, KT, v4f{0.f, 0.f, 0.f, 0.f});
      const int c = c0 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + 4 * (lane >> 4) + q;
        if (row < ROWS) {
          const int g = row / (HI * HI), pq = row - g * HI * HI;
          dprev[(g * CIN + c) * HI * HI + pq] = acc[q];
        }
      }
    }
  }
  __syncthreads();
}

template <bool BF16, int G, int C, int F, int NC>
__global__ __launch_bounds__(kEncThreads) void k_encoder_bwd(const float* __restrict__ x, int n,
                                                             const float* __restrict__ dfeat,
                                                             const float* __restrict__ W0, const float* __restrict__ W1,
                                                             const float* __restrict__ W2,
                                                             const float* __restrict__ h0, const float* __restrict__ h1,
                                                             const float* __restrict__ h2, long long W_off0,
                                                             long long b_off0, long long W_off1, long long b_off1,
                                                             long long W_off2, long long b_off2, long long enc_total,
                                                             float* __restrict__ part) {
  constexpr int BIG = G * F * 49 > G * C * 256 ? G * F * 49 : G * C * 256;
  __shared__ float ld_a[G * F * 49];    // gradient at the current layer's output
  __shared__ float ld_b[G * F * 49];    // gradient at its input
  __shared__ float ld_in[BIG];          // the current layer's input activation
  const int img0 = blockIdx.x * G;
  const int gn = n - img0 < G ? n - img0 : G;
  float* pp = part + (long long)blockIdx.x * enc_total;
  constexpr int FL = NC > 2 ? 9 : 25;   // pixels of the last layer's output
  const float* hl = NC > 2 ? h2 : h1;
  for (int e = threadIdx.x; e < G * F * FL; e += kEncThreads) {
    const int g = e / (F * FL);
    ld_a[e] = g < gn ? dfeat[(long long)img0 * F * FL + e] : 0.f;
  }
  float* dcur = ld_a;
  float* dnext = ld_b;
  if constexpr (NC > 2) {
    for (int e = threadIdx.x; e < G * F * 25; e += kEncThreads) {
      const int g = e / (F * 25);
      ld_in[e] = g < gn ? h1[(long long)img0 * F * 25 + e] : 0.f;
    }
    __syncthreads();
    conv_layer_bwd<BF16, G, F, F, 5, 3, 1, true>(dcur, hl + (long long)img0 * F * 9, ld_in, W2, pp + W_off2,
                                                 pp + b_off2, dnext, gn);
    float* t = dcur; dcur = dnext; dnext = t;
  }
  for (int e = threadIdx.x; e < G * F * 49; e += kEncThreads) {
    const int g = e / (F * 49);
    ld_in[e] = g < gn ? h0[(long long)img0 * F * 49 + e] : 0.f;
  }
  __syncthreads();
  conv_layer_bwd<BF16, G, F, F, 7, 5, 1, true>(dcur, h1 + (long long)img0 * F * 25, ld_in, W1, pp + W_off1,
                                               pp + b_off1, dnext, gn);
  { float* t = dcur; dcur = dnext; dnext = t; }
  for (int e = threadIdx.x; e < G * C * 256; e += kEncThreads) {
    const int g = e / (C * 256);
    ld_in[e] = g < gn ? x[(long long)img0 * C * 256 + e] : 0.f;
  }
  __syncthreads();
  conv_layer_bwd<BF16, G, C, F, 16, 7, 2, false>(dcur, h0 + (long long)img0 * F * 49, ld_in, W0, pp + W_off0,
                                                 pp + b_off0, nullptr, gn);
}

// grad[e] = sum over workgroups (in order) of part[wg][e]
__global__ __launch_bounds__(256) void k_enc_reduce(const float* __restrict__ part, int nwg, long long total,
                                                    float* __restrict__ grad) {
  __shared__ float sh[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e = (long long)blockIdx.x * 64 + lane;
  float v = 0.f;
  if (e < total)
    for (int w = wave; w < nwg; w += 4) v += part[(long long)w * total + e];
  sh[wave][lane] = v;
  __syncthreads();
  if (wave == 0 && e < total) grad[e] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

// ---------------------------------------------------------------- launchers
constexpr int kEncG = 2;

template <bool BF16, int C, int F, int NC>
static int enc_fwd_t(const float* x, int n, const float* const* W, const float* const* b, float* const* h,
                     hipStream_t st) {
  const int nwg = cdiv(n, kEncG);
  k_encoder_fwd<BF16, kEncG, C, F, NC><<<nwg, kEncThreads, 0, st>>>(x, n, W[0], b[0], W[1], b[1], NC > 2 ? W[2] : W[1],
                                                                    NC > 2 ? b[2] : b[1], h[0], h[1],
                                                                    NC > 2 ? h[2] : h[1]);
  return launch_status("encoder_fwd");
}

template <bool BF16, int C, int F, int NC>
static int enc_bwd_t(const float* x, int n, const float* dfeat, const float* const* W, const float* const* h,
                     const long long* Woff, const long long* boff, long long total, float* part, float* grad,
                     hipStream_t st) {
  const int nwg = cdiv(n, kEncG);
  k_encoder_bwd<BF16, kEncG, C, F, NC><<<nwg, kEncThreads, 0, st>>>(
      x, n, dfeat, W[0], W[1], NC > 2 ? W[2] : W[1], h[0], h[1], NC > 2 ? h[2] : h[1], Woff[0], boff[0], Woff[1],
      boff[1], NC > 2 ? Woff[2] : 0, NC > 2 ? boff[2] : 0, total, part);
  SQ_TRY(launch_status("encoder_bwd"));
  k_enc_reduce<<<cdiv(total, 64), 256, 0, st>>>(part, nwg, total, grad);
  return launch_status("encoder_reduce");
}

bool encoder_fused_ok(int C, int F, int n_conv, int side) {
  return side == 16 && ((C == 9 && F == 32 && n_conv == 3) || (C == 3 && F == 16 && n_conv == 2));
}

size_t encoder_fused_part_floats(int n, long long enc_total) { return (size_t)cdiv(n, kEncG) * enc_total; }

int encoder_fused_fwd(int bf16, int C, int F, int n_conv, const float* x, int n, const float* const* W,
                      const float* const* b, float* const* h, hipStream_t st) {
  if (n <= 0) return SQ_OK;
  if (C == 9 && F == 32 && n_conv == 3)
    return bf16 ? enc_fwd_t<true, 9, 32, 3>(x, n, W, b, h, st) : enc_fwd_t<false, 9, 32, 3>(x, n, W, b, h, st);
  return bf16 ? enc_fwd_t<true, 3, 16, 2>(x, n, W, b, h, st) : enc_fwd_t<false, 3, 16, 2>(x, n, W, b, h, st);
}

int encoder_fused_bwd(int bf16, int C, int F, int n_conv, const float* x, int n, const float* dfeat,
                      const float* const* W, const float* const* h, const long long* Woff, const long long* boff,
                      long long total, float* part, float* grad, hipStream_t st) {
  if (n <= 0) return SQ_OK;
  if (C == 9 && F == 32 && n_conv == 3)
    return bf16 ? enc_bwd_t<true, 9, 32, 3>(x, n, dfeat, W, h, Woff, boff, total, part, grad, st)
                : enc_bwd_t<false, 9, 32, 3>(x, n, dfeat, W, h, Woff, boff, total, part, grad, st);
  return bf16 ? enc_bwd_t<true, 3, 16, 2>(x, n, dfeat, W, h, Woff, boff, total, part, grad, st)
              : enc_bwd_t<false, 3, 16, 2>(x, n, dfeat, W, h, Woff, boff, total, part, grad, st);
}

}  // namespace sq
