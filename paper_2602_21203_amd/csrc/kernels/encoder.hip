// Fused conv encoder for 16x16 squinted images (Sec. IV Encoder Design Choices),
// and, in the bfloat16 form, for the 32x32 input of the camera-resolution
// analysis (Sec. VI): 32 -> 15 -> 13 -> 11 with one image per backward workgroup.
// 3x3 valid convolutions, the first with stride 2, ReLU after each.
//
// Data layout.  Inside a workgroup every activation and gradient lives in LDS
// channel-innermost ([image][y][x][channel], pixels padded to a multiple of 16
// channels plus 4 floats so that 16-byte reads of neighbouring pixels spread
// over the banks).  A small preparation kernel rewrites the conv weights into
// the two orders the contractions read with 16-byte loads: [f][tap][c] for the
// forward and [tap][c][f] for the input gradient (bfloat16-rounded in the
// bfloat16 form).
//
// FP32 form: contractions run on v_mfma_f32_16x16x4_f32.  In a chunk of 16
// consecutive channels of one tap, lane (li, lq) loads channels 4*lq .. 4*lq + 3
// of its row and of its column with one 16-byte load each and feeds them to four
// consecutive MFMA steps, so the gather costs one LDS read and one global read
// per four steps, at addresses fixed at compile time up to a per-lane base.
//
// bfloat16 form (the k_*_b kernels below): activations, inputs and gradients
// are held in LDS as bfloat16 (half the footprint, so more workgroups share a
// CU) and contracted with v_mfma_f32_16x16x32_bf16, FP32 accumulation.  Every
// operand is rounded to bfloat16 once, when it is written to LDS or prepared;
// bias gradients are summed from the unrounded FP32 values.  A 32-wide k chunk
// is one tap of 32 channels, or two taps of 16 (padded) channels, a tenth
// phantom tap contributing zero.
//
// Forward: a workgroup owns G images.  Layer outputs go to LDS (next layer's
// operand) and to HBM (FP32; [n][pixel][F] for the inner layers, NCHW for the
// last one, which is the flattened feature vector).
//
// Backward: per layer, from the gradient at its post-ReLU output (masked by
// output > 0): the bias sum, the weight gradient of the G images (contraction
// over their output pixels, whose LDS offsets come from a per-layer table) and,
// above the first layer, the input gradient (a transposed convolution over a
// zero-bordered copy of the gradient, masked by the layer's input > 0 on the
// way out).  Each workgroup writes its partial encoder gradient; a second
// kernel adds the partials in workgroup order, so the result is deterministic.
#include "../common.h"
#include "bf16.h"
#include "sample.h"

namespace sq {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int r16(int x) { return (x + 15) / 16 * 16; }
__host__ __device__ constexpr int enc_in(int l) { return l == 0 ? 16 : (l == 1 ? 7 : (l == 2 ? 5 : 3)); }
__host__ __device__ constexpr int enc_out(int l) { return l == 0 ? 7 : (l == 1 ? 5 : (l == 2 ? 3 : 1)); }

// layer l of an encoder with C input channels and F filters
template <int C, int F, int l> struct LG {
  static constexpr int CIN = l == 0 ? C : F;
  static constexpr int CP = r16(CIN);         // channels per pixel held in LDS (zero padded)
  static constexpr int PS = CP + 4;           // LDS floats per input pixel
  static constexpr int HI = enc_in(l), HO = enc_out(l), S = l == 0 ? 2 : 1;
  static constexpr int P = HO * HO;           // output pixels per image
  static constexpr int K = CIN * 9;           // weights per filter
  static constexpr int DS = HO + 4;           // side of the zero-bordered output-gradient buffer
  static constexpr int WF = F * 9 * CP;       // prepared forward weights [f][tap][CP]
  static constexpr int WB = l == 0 ? 0 : 9 * CIN * F;   // prepared input-gradient weights [tap][c][f]
};

// offsets of the prepared weight blocks
template <int C, int F, int NC> struct EncPrep {
  static constexpr int F0 = 0;
  static constexpr int F1 = F0 + LG<C, F, 0>::WF;
  static constexpr int F2 = F1 + LG<C, F, 1>::WF;
  static constexpr int B1 = F2 + (NC > 2 ? LG<C, F, 2>::WF : 0);
  static constexpr int B2 = B1 + LG<C, F, 1>::WB;
  static constexpr int TOTAL = B2 + (NC > 2 ? LG<C, F, 2>::WB : 0);
};

__device__ __forceinline__ float rnd(float v, bool on) { return on ? bf16_round(v) : v; }

__device__ __forceinline__ v4f mma4(const f4v& a, const f4v& b, v4f acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
  return acc;
}

// ---------------------------------------------------------------- weight preparation
struct EncW {
  const float* W[3];
};

template <int C, int F, int NC>
__global__ __launch_bounds__(256) void k_enc_prep(EncW w, float* __restrict__ wp, int bf16) {
  using E = EncPrep<C, F, NC>;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < E::TOTAL; e += gridDim.x * 256) {
    float v;
    if (e < E::B1) {                       // forward order [f][tap][CP]
      int l, o, cin, cp;
      if (e < E::F1) { l = 0; o = e; cin = C; cp = LG<C, F, 0>::CP; }
      else if (e < E::F2) { l = 1; o = e - E::F1; cin = F; cp = LG<C, F, 1>::CP; }
      else { l = 2; o = e - E::F2; cin = F; cp = LG<C, F, 2>::CP; }
      const int f = o / (9 * cp), r = o - f * 9 * cp, tap = r / cp, c = r - tap * cp;
      v = c < cin ? w.W[l][(f * cin + c) * 9 + tap] : 0.f;
    } else {                               // input-gradient order [tap][c][f]
      const int l = e < E::B2 ? 1 : 2;
      const int o = e - (l == 1 ? E::B1 : E::B2);
      const int tap = o / (F * F), r = o - tap * F * F, c = r / F, f = r - c * F;
      v = w.W[l][(f * F + c) * 9 + tap];
    }
    if (bf16) reinterpret_cast<uint16_t*>(wp)[e] = bf16_bits(v);   // packed bfloat16 elements
    else wp[e] = v;
  }
}

// ---------------------------------------------------------------- forward
// One conv layer of G images: in [G][HI][HI][PS] (LDS) -> post-ReLU
// out_lds [G][HO][HO][F + 4] (the next layer's operand, rounded in the bfloat16
// form) and out_g (FP32; [img][pixel][F], or NCHW for the last layer).
template <bool BF16, int G, int C, int F, int l, bool TO_LDS, bool LAST, int NT>
__device__ void conv_fwd_layer(const float* in, float* out_lds, const float* __restrict__ wf,
                               const float* __restrict__ bias, float* __restrict__ out_g, int gn) {
  using Y = LG<C, F, l>;
  constexpr int ROWS = G * Y::P, RT = (ROWS + 15) / 16, CT = F / 16, NW = NT / 64;
  constexpr int PSO = F + 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  for (int t = wave; t < RT * CT; t += NW) {
    const int rt = t / CT, ct = t - rt * CT;
    const int r0 = rt * 16, c0 = ct * 16;
    const int row = min(r0 + li, ROWS - 1);
    const int g = row / Y::P, p = row - g * Y::P, oy = p / Y::HO, ox = p - oy * Y::HO;
    const float* ap = in + ((g * Y::HI + oy * Y::S) * Y::HI + ox * Y::S) * Y::PS + 4 * lq;
    const float* bp = wf + (c0 + li) * 9 * Y::CP + 4 * lq;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
      for (int cg = 0; cg < Y::CP / 16; ++cg) {
        const f4v a = *reinterpret_cast<const f4v*>(ap + (ky * Y::HI + kx) * Y::PS + 16 * cg);
        const f4v b = *reinterpret_cast<const f4v*>(__builtin_assume_aligned(bp + tap * Y::CP + 16 * cg, 16));
        acc = mma4(a, b, acc);
      }
    }
    const int f = c0 + li;
    const float bv = bias[f];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 4 * lq + q;
      if (r < ROWS) {
        const int gg = r / Y::P, pp = r - gg * Y::P;
        const float v = fmaxf(acc[q] + bv, 0.f);
        if constexpr (TO_LDS) out_lds[(gg * Y::P + pp) * PSO + f] = rnd(v, BF16);
        if (gg < gn) {
          if constexpr (LAST) out_g[((long long)gg * F + f) * Y::P + pp] = v;
          else out_g[((long long)gg * Y::P + pp) * F + f] = v;
        }
      }
    }
  }
}

template <bool BF16, int G, int C, int F, int NC, int NT>
__global__ __launch_bounds__(NT) void k_encoder_fwd(const float* __restrict__ x, int n, const float* __restrict__ wp,
                                                    const float* __restrict__ b0, const float* __restrict__ b1,
                                                    const float* __restrict__ b2, float* __restrict__ h0,
                                                    float* __restrict__ h1, float* __restrict__ h2) {
  using L0 = LG<C, F, 0>;
  using L1 = LG<C, F, 1>;
  using E = EncPrep<C, F, NC>;
  constexpr int X = G * 256 * L0::PS, A0 = G * L0::P * (F + 4), A1 = NC > 2 ? G * L1::P * (F + 4) : 4;
  __shared__ __attribute__((aligned(16))) float lx[X];
  __shared__ __attribute__((aligned(16))) float la0[A0];
  __shared__ __attribute__((aligned(16))) float la1[A1];
  const int img0 = blockIdx.x * G;
  const int gn = n - img0 < G ? n - img0 : G;
  // images of this group, NCHW -> [g][pixel][channel]; absent images and padding channels read as zero
  for (int e = threadIdx.x; e < G * C * 256; e += NT) {
    const int g = e / (C * 256), r = e - g * C * 256, c = r >> 8, pix = r & 255;
    lx[(g * 256 + pix) * L0::PS + c] = g < gn ? rnd(x[(long long)img0 * C * 256 + e], BF16) : 0.f;
  }
  for (int e = threadIdx.x; e < G * 256 * (L0::CP - C); e += NT) {
    const int gp = e / (L0::CP - C), c = C + e - gp * (L0::CP - C);
    lx[gp * L0::PS + c] = 0.f;
  }
  __syncthreads();
  conv_fwd_layer<BF16, G, C, F, 0, true, false, NT>(lx, la0, wp + E::F0, b0, h0 + (long long)img0 * F * L0::P, gn);
  __syncthreads();
  if constexpr (NC > 2) {
    conv_fwd_layer<BF16, G, C, F, 1, true, false, NT>(la0, la1, wp + E::F1, b1, h1 + (long long)img0 * F * L1::P, gn);
    __syncthreads();
    conv_fwd_layer<BF16, G, C, F, 2, false, true, NT>(la1, nullptr, wp + E::F2, b2,
                                                      h2 + (long long)img0 * F * LG<C, F, 2>::P, gn);
  } else {
    conv_fwd_layer<BF16, G, C, F, 1, false, true, NT>(la0, nullptr, wp + E::F1, b1, h1 + (long long)img0 * F * L1::P,
                                                      gn);
  }
}

// ---------------------------------------------------------------- backward
// Gradient buffers: layer l's output gradient D_l as [G][DS][DS][F + 4] with a
// zero border of 2 (interior pixel (y, x) at (y + 2, x + 2)).

// From D_l (interior filled, border zero): bias partial, bfloat16 rounding of
// D_l in that form, weight partial over the images' output pixels.  `in` is the
// layer's input [G][HI][HI][PS].
template <bool BF16, int G, int C, int F, int l, int NT>
__device__ void conv_bwd_weights(float* D, const float* in, int2* qtab, float* __restrict__ partW,
                                 float* __restrict__ partb) {
  using Y = LG<C, F, l>;
  constexpr int PSF = F + 4;
  constexpr int NPOS = G * Y::P, NQ = (NPOS + 3) / 4 * 4, NW = NT / 64;
  // bias: thread f sums its channel over the images' pixels in order (unrounded)
  if (threadIdx.x < F) {
    const int f = threadIdx.x;
    float sb = 0.f;
    for (int g = 0; g < G; ++g)
      for (int p = 0; p < Y::P; ++p) {
        const int oy = p / Y::HO, ox = p - oy * Y::HO;
        sb += D[((g * Y::DS + oy + 2) * Y::DS + ox + 2) * PSF + f];
      }
    partb[f] = sb;
  }
  // contraction table: output pixel q -> (offset in D, offset of its input patch
  // origin); the pad entries point at a zero border pixel of D
  for (int q = threadIdx.x; q < NQ; q += NT) {
    int2 e = make_int2(0, 0);
    if (q < NPOS) {
      const int g = q / Y::P, p = q - g * Y::P, oy = p / Y::HO, ox = p - oy * Y::HO;
      e.x = ((g * Y::DS + oy + 2) * Y::DS + ox + 2) * PSF;
      e.y = ((g * Y::HI + oy * Y::S) * Y::HI + ox * Y::S) * Y::PS;
    }
    qtab[q] = e;
  }
  __syncthreads();
  if constexpr (BF16) {
    for (int e = threadIdx.x; e < G * Y::DS * Y::DS * PSF; e += NT) D[e] = bf16_round(D[e]);
    __syncthreads();
  }
  // weights: rows f (F / 16 tiles), columns kc = c * 9 + tap (the parameter order, so
  // a tile's stores are 16 consecutive floats per row), contraction over output pixels
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  constexpr int RT = F / 16, CT = (Y::K + 15) / 16;
  for (int t = wave; t < RT * CT; t += NW) {
    const int rt = t / CT, ct = t - rt * CT;
    const int f0 = rt * 16, k0 = ct * 16;
    const int kc = min(k0 + li, Y::K - 1);
    const int c = kc / 9, tap = kc - 9 * c, ky = tap / 3, kx = tap - 3 * ky;
    const float* ap = D + f0 + li;
    const float* bp = in + (ky * Y::HI + kx) * Y::PS + c;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int s = 0; s < NQ / 4; ++s) {
      const int2 e = qtab[4 * s + lq];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[e.x], bp[e.y], acc, 0, 0, 0);
    }
    const int kk = k0 + li;
    if (kk < Y::K) {
#pragma unroll
      for (int q = 0; q < 4; ++q) partW[(f0 + 4 * lq + q) * Y::K + kk] = acc[q];
    }
  }
}

// Input gradient of layer l >= 1 from D_l (rounded in the bfloat16 form):
// E[g][iy][ix][c] = sum_{tap, f} D_l[g][iy - ky][ix - kx][f] W[f][c][ky][kx],
// masked by the layer's input (hin = layer l-1's output, [img][pixel][F]) > 0
// and written into the interior of Dn (zero-bordered [G][HI + 4][HI + 4][F + 4]).
template <int G, int C, int F, int l, int NT>
__device__ void conv_bwd_input(const float* D, const float* __restrict__ wb, const float* __restrict__ hin, float* Dn,
                               int gn) {
  using Y = LG<C, F, l>;
  static_assert(l >= 1, "input gradients are needed above the first layer only");
  constexpr int PSF = F + 4, DSN = Y::HI + 4;
  constexpr int ROWS = G * Y::HI * Y::HI, RT = (ROWS + 15) / 16, CT = F / 16, NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  for (int t = wave; t < RT * CT; t += NW) {
    const int rt = t / CT, ct = t - rt * CT;
    const int r0 = rt * 16, c0 = ct * 16;
    const int row = min(r0 + li, ROWS - 1);
    const int g = row / (Y::HI * Y::HI), pq = row - g * Y::HI * Y::HI, iy = pq / Y::HI, ix = pq - iy * Y::HI;
    const float* ap = D + ((g * Y::DS + iy + 2) * Y::DS + ix + 2) * PSF + 4 * lq;
    const float* bp = wb + (c0 + li) * F + 4 * lq;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
      for (int fg = 0; fg < F / 16; ++fg) {
        const f4v a = *reinterpret_cast<const f4v*>(ap - (ky * Y::DS + kx) * PSF + 16 * fg);
        const f4v b = *reinterpret_cast<const f4v*>(__builtin_assume_aligned(bp + tap * F * F + 16 * fg, 16));
        acc = mma4(a, b, acc);
      }
    }
    const int c = c0 + li;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 4 * lq + q;
      if (r < ROWS) {
        const int gg = r / (Y::HI * Y::HI), pp = r - gg * Y::HI * Y::HI, yy = pp / Y::HI, xx = pp - yy * Y::HI;
        const bool live = gg < gn && hin[((long long)gg * Y::HI * Y::HI + pp) * F + c] > 0.f;
        Dn[((gg * DSN + yy + 2) * DSN + xx + 2) * PSF + c] = live ? acc[q] : 0.f;
      }
    }
  }
}

struct EncOffs {
  long long W[3], b[3];
};

template <bool BF16, int G, int C, int F, int NC, int NT>
__global__ __launch_bounds__(NT) void k_encoder_bwd(const float* __restrict__ x, int n,
                                                    const float* __restrict__ dfeat, const float* __restrict__ wp,
                                                    const float* __restrict__ h0, const float* __restrict__ h1,
                                                    const float* __restrict__ h2, EncOffs off, long long enc_total,
                                                    float* __restrict__ part) {
  using L0 = LG<C, F, 0>;
  using L1 = LG<C, F, 1>;
  using LL = LG<C, F, NC - 1>;
  using E = EncPrep<C, F, NC>;
  constexpr int PSF = F + 4;
  constexpr int SZ0 = G * L0::DS * L0::DS * PSF;                                  // D_0
  constexpr int SZ1 = G * L1::DS * L1::DS * PSF;                                  // D_1
  constexpr int SZ2 = NC > 2 ? G * LG<C, F, 2>::DS * LG<C, F, 2>::DS * PSF : 4;   // D_2
  // region r0 holds D_2 first and D_0 last (never live together); r1 holds D_1
  constexpr int R0 = SZ0 > SZ2 ? SZ0 : SZ2;
  constexpr int IN0 = G * 256 * L0::PS, IN1 = G * L1::HI * L1::HI * L1::PS;
  constexpr int RIN = IN0 > IN1 ? IN0 : IN1;
  constexpr int NQ = (G * L0::P + 3) / 4 * 4;
  __shared__ __attribute__((aligned(16))) float r0[R0];
  __shared__ __attribute__((aligned(16))) float r1[SZ1];
  __shared__ __attribute__((aligned(16))) float rin[RIN];
  __shared__ int2 qtab[NQ];
  const int img0 = blockIdx.x * G;
  const int gn = n - img0 < G ? n - img0 : G;
  float* pp = part + (long long)blockIdx.x * enc_total;

  // D_{NC-1}: zero, then the upstream gradient (NCHW) masked by the output > 0 into the interior
  float* Dl = NC > 2 ? r0 : r1;
  for (int e = threadIdx.x; e < (NC > 2 ? SZ2 : SZ1); e += NT) Dl[e] = 0.f;
  __syncthreads();
  {
    const float* hl = NC > 2 ? h2 : h1;
    for (int e = threadIdx.x; e < G * F * LL::P; e += NT) {
      const int g = e / (F * LL::P), r = e - g * F * LL::P, f = r / LL::P, p = r - f * LL::P;
      const int oy = p / LL::HO, ox = p - oy * LL::HO;
      const long long gi = (long long)img0 * F * LL::P + e;
      const float v = (g < gn && hl[gi] > 0.f) ? dfeat[gi] : 0.f;
      Dl[((g * LL::DS + oy + 2) * LL::DS + ox + 2) * PSF + f] = v;
    }
  }
  if constexpr (NC > 2) {
    using L2 = LG<C, F, 2>;
    // layer 2: input h1 ([img][pixel][F] -> [g][pixel][PS]); D_2 in r0, D_1 -> r1
    for (int e = threadIdx.x; e < G * L2::HI * L2::HI * F; e += NT) {
      const int gp = e / F, c = e - gp * F, g = gp / (L2::HI * L2::HI);
      rin[gp * L2::PS + c] = g < gn ? rnd(h1[(long long)img0 * L2::HI * L2::HI * F + e], BF16) : 0.f;
    }
    for (int e = threadIdx.x; e < SZ1; e += NT) r1[e] = 0.f;
    __syncthreads();
    conv_bwd_weights<BF16, G, C, F, 2, NT>(r0, rin, qtab, pp + off.W[2], pp + off.b[2]);
    __syncthreads();
    conv_bwd_input<G, C, F, 2, NT>(r0, wp + E::B2, h1 + (long long)img0 * L2::HI * L2::HI * F, r1, gn);
    __syncthreads();
  }
  // layer 1: input h0; D_1 in r1, D_0 -> r0
  for (int e = threadIdx.x; e < G * L1::HI * L1::HI * F; e += NT) {
    const int gp = e / F, c = e - gp * F, g = gp / (L1::HI * L1::HI);
    rin[gp * L1::PS + c] = g < gn ? rnd(h0[(long long)img0 * L1::HI * L1::HI * F + e], BF16) : 0.f;
  }
  for (int e = threadIdx.x; e < SZ0; e += NT) r0[e] = 0.f;
  __syncthreads();
  conv_bwd_weights<BF16, G, C, F, 1, NT>(r1, rin, qtab, pp + off.W[1], pp + off.b[1]);
  __syncthreads();
  conv_bwd_input<G, C, F, 1, NT>(r1, wp + E::B1, h0 + (long long)img0 * L1::HI * L1::HI * F, r0, gn);
  __syncthreads();
  // layer 0: input x (NCHW -> [g][pixel][channel], padding channels zero); D_0 in r0
  for (int e = threadIdx.x; e < G * C * 256; e += NT) {
    const int g = e / (C * 256), r = e - g * C * 256, c = r >> 8, pix = r & 255;
    rin[(g * 256 + pix) * L0::PS + c] = g < gn ? rnd(x[(long long)img0 * C * 256 + e], BF16) : 0.f;
  }
  for (int e = threadIdx.x; e < G * 256 * (L0::CP - C); e += NT) {
    const int gp = e / (L0::CP - C), c = C + e - gp * (L0::CP - C);
    rin[gp * L0::PS + c] = 0.f;
  }
  __syncthreads();
  conv_bwd_weights<BF16, G, C, F, 0, NT>(r0, rin, qtab, pp + off.W[0], pp + off.b[0]);
}

// grad[e] = sum over workgroups (in order) of part[wg][e]: four consecutive
// elements per lane, the workgroup rows split over the four waves by residue,
// the four wave sums added in wave order
__global__ __launch_bounds__(256) void k_enc_reduce(const float* __restrict__ part, int nwg, long long total,
                                                    float* __restrict__ grad) {
  __shared__ f4v sh[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e = ((long long)blockIdx.x * 64 + lane) * 4;
  const bool vec = total % 4 == 0 && e + 4 <= total;
  f4v v = f4v{0.f, 0.f, 0.f, 0.f};
  if (vec) {
#pragma unroll 8
    for (int w = wave; w < nwg; w += 4)
      v += *reinterpret_cast<const f4v*>(__builtin_assume_aligned(part + (long long)w * total + e, 16));
  } else {
    for (int w = wave; w < nwg; w += 4)
      for (int j = 0; j < 4; ++j)
        if (e + j < total) v[j] += part[(long long)w * total + e + j];
  }
  sh[wave][lane] = v;
  __syncthreads();
  if (wave == 0) {
    const f4v s = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
    for (int j = 0; j < 4; ++j)
      if (e + j < total) grad[e + j] = s[j];
  }
}

// ---------------------------------------------------------------- bfloat16 form
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// layer geometry with bfloat16 storage: PS elements per LDS pixel (16-byte aligned),
// TPM taps per 32-wide k chunk, NM chunks per 3x3 contraction
// on SD x SD images: SD -> (SD - 3) / 2 + 1 (stride 2) -> then 2 less per layer
template <int C, int F, int l, int SD> struct LB {
  static constexpr int CIN = l == 0 ? C : F;
  static constexpr int CP = r16(CIN);
  static constexpr int PS = CP + 8;
  static constexpr int O0 = (SD - 3) / 2 + 1;
  static constexpr int HI = l == 0 ? SD : O0 - 2 * (l - 1), HO = l == 0 ? O0 : HI - 2, S = l == 0 ? 2 : 1;
  static constexpr int P = HO * HO;
  static constexpr int K = CIN * 9;
  static constexpr int DS = HO + 4;
  static constexpr int TPM = 32 / CP;
  static constexpr int NM = (9 + TPM - 1) / TPM;
  static_assert(CP == 16 || CP == 32, "16 or 32 (padded) channels per tap");
};

__device__ __forceinline__ v4f mma_b(const bf16x8& a, const bf16x8& b, v4f acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// Workgroup barrier for LDS hand-offs only: the thread's LDS operations complete
// before it, while its global loads stay in flight (no global memory is written
// and read back by other threads inside these kernels).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// the chunk's tap and channel offset for lane group lq (tap 9 is the phantom tap
// of an odd count: its weight operand is zero, its input read is clamped to tap 8)
template <int TPM>
__device__ __forceinline__ void chunk_tap(int mi, int lq, int& tap, int& off) {
  if constexpr (TPM == 1) { tap = mi; off = 8 * lq; }
  else { tap = 2 * mi + (lq >> 1); off = 8 * (lq & 1); }
}

// The weight operand of one column tile (16 filters from c0) of forward layer l,
// as this lane's MFMA fragments of every k chunk.  When the workgroup's wave count
// is a multiple of the layer's column tiles, a wave only ever meets one column
// tile, so all of a wave's weight fragments can be requested up front.
template <int C, int F, int l, int SD>
struct WFrag {
  using Y = LB<C, F, l, SD>;
  bf16x8 b[Y::NM];
  float bias;
  __device__ __forceinline__ void load(const __bf16* __restrict__ wf, const float* __restrict__ bs, int c0) {
    const int lane = threadIdx.x & 63, li = lane & 15, lq = lane >> 4;
    const __bf16* bp = wf + (c0 + li) * 9 * Y::CP;
#pragma unroll
    for (int mi = 0; mi < Y::NM; ++mi) {
      int tap, off;
      chunk_tap<Y::TPM>(mi, lq, tap, off);
      const int tc = tap < 9 ? tap : 8;
      b[mi] = *reinterpret_cast<const bf16x8*>(__builtin_assume_aligned(bp + tc * Y::CP + off, 16));
      if (tap > 8) b[mi] = bf16x8{};
    }
    bias = bs[c0 + li];
  }
};

// forward layer l of G images: in [G][HI][HI][PS] (bfloat16, LDS) -> post-ReLU
// out_lds [G][HO][HO][F + 8] (bfloat16) and out_g (FP32, as the FP32 form).
// w: the wave's weight fragments when PRE (its one column tile), else read per tile.
template <int G, int C, int F, int l, int SD, bool TO_LDS, bool LAST, int NT, bool PRE>
__device__ void conv_fwd_layer_b(const __bf16* in, __bf16* out_lds, const __bf16* __restrict__ wf,
                                 const float* __restrict__ bias, float* __restrict__ out_g, int gn,
                                 const WFrag<C, F, l, SD>& w, float* out_lds_f = nullptr,
                                 uint16_t* __restrict__ out_h = nullptr) {
  using Y = LB<C, F, l, SD>;
  constexpr int ROWS = G * Y::P, RT = (ROWS + 15) / 16, CT = F / 16, NW = NT / 64;
  constexpr int PSO = F + 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  for (int t = wave; t < RT * CT; t += NW) {
    const int rt = t / CT, ct = t - rt * CT;
    const int r0 = rt * 16, c0 = ct * 16;
    const int row = min(r0 + li, ROWS - 1);
    const int g = row / Y::P, p = row - g * Y::P, oy = p / Y::HO, ox = p - oy * Y::HO;
    const __bf16* ap = in + ((g * Y::HI + oy * Y::S) * Y::HI + ox * Y::S) * Y::PS;
    WFrag<C, F, l, SD> wt;
    if constexpr (!PRE) wt.load(wf, bias, c0);
    const WFrag<C, F, l, SD>& ww = PRE ? w : wt;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mi = 0; mi < Y::NM; ++mi) {
      int tap, off;
      chunk_tap<Y::TPM>(mi, lq, tap, off);
      const int tc = tap < 9 ? tap : 8, ky = tc / 3, kx = tc - 3 * ky;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap + (ky * Y::HI + kx) * Y::PS + off);
      acc = mma_b(a, ww.b[mi], acc);
    }
    const int f = c0 + li;
    const float bv = ww.bias;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 4 * lq + q;
      if (r < ROWS) {
        const int gg = r / Y::P, pp = r - gg * Y::P;
        const float v = fmaxf(acc[q] + bv, 0.f);
        if constexpr (TO_LDS) out_lds[(gg * Y::P + pp) * PSO + f] = (__bf16)v;
        if constexpr (LAST) out_lds_f[(gg * F + f) * Y::P + pp] = v;   // NCHW, stored below
        else if (gg < gn) out_g[((long long)gg * Y::P + pp) * F + f] = v;
      }
    }
  }
  if constexpr (LAST) {
    // the feature rows of the workgroup's images are contiguous in NCHW order
    lds_barrier();
    for (int e = threadIdx.x; e < gn * F * Y::P; e += NT) {
      out_g[e] = out_lds_f[e];
      if (out_h) out_h[e] = bf16_bits(out_lds_f[e]);
    }
  }
}

// SQK > 0: the launch also draws the minibatch and squints its frames (factor
// SQK, uint8 HWC frames of side SD * SQK; SQK = 1: the block means stored in a
// ring at insertion): the first `lead` workgroups take the draw's items (as in
// the squint launch), and image workgroup i computes replay row i of the draw
// itself (obs rows, then next_obs rows), sums each output pixel's SQK x SQK
// block per channel (thread p owns pixel p), and writes x = sum / (255 SQK^2) -
// 0.5 both to xout (FP32 CHW, for the backward) and, rounded, to the first
// layer's LDS input: the separate draw / squint launches and the round trip of x
// disappear.  The arithmetic is the squint kernels'.
template <int G, int C, int F, int NC, int SD, int NT, int SQK = 0>
__global__ __launch_bounds__(NT) void k_encoder_fwd_b(const float* __restrict__ x, int n, const __bf16* __restrict__ wp,
                                                      const float* __restrict__ b0, const float* __restrict__ b1,
                                                      const float* __restrict__ b2, float* __restrict__ h0,
                                                      float* __restrict__ h1, float* __restrict__ h2,
                                                      uint16_t* __restrict__ hh, const uint8_t* __restrict__ obs,
                                                      const uint8_t* __restrict__ next_obs, SampleArgs sa, int lead,
                                                      float* __restrict__ xout) {
  using L0 = LB<C, F, 0, SD>;
  using L1 = LB<C, F, 1, SD>;
  using E = EncPrep<C, F, NC>;
  constexpr int X = G * SD * SD * L0::PS, A0 = G * L0::P * (F + 8), A1 = NC > 2 ? G * L1::P * (F + 8) : 8;
  constexpr int NW = NT / 64, CT = F / 16;
  constexpr bool PRE = NW % CT == 0;   // each wave meets one column tile per layer
  __shared__ __attribute__((aligned(16))) __bf16 lx[X];
  __shared__ __attribute__((aligned(16))) __bf16 la0[A0];
  __shared__ __attribute__((aligned(16))) __bf16 la1[A1];
  if constexpr (SQK > 0) {
    if ((int)blockIdx.x < lead) {
      const long long t = (long long)blockIdx.x * NT + threadIdx.x;
      if (t < sample_items(sa.B, sa.A, sa.S)) sample_item(sa, t);
      return;
    }
  }
  const int img0 = ((int)blockIdx.x - (SQK > 0 ? lead : 0)) * G;
  const int gn = n - img0 < G ? n - img0 : G;
  // the images, then every layer's weight fragments of this wave, all requested up front
  constexpr int RX = SQK > 0 ? 1 : (G * C * SD * SD + NT - 1) / NT;
  constexpr int SEG = SQK * C;   // bytes of one source block row (squint form)
  constexpr int NWD = SQK > 1 ? SQK * SEG / 4 : (SQK == 1 ? C : 1);
  float xv[RX];
  unsigned fw[NWD];   // the block rows as 32-bit words (SQK > 1), or the pixel's C bytes (SQK = 1)
  if constexpr (SQK > 0) {
    static_assert(G == 1 && NT == SD * SD && (SQK == 1 || SEG % 4 == 0),
                  "one thread per output pixel, 32-bit block rows");
    const int p = threadIdx.x, y = p / SD, xq = p - y * SD;
    constexpr int Wsrc = SD * SQK;
    const bool second = img0 >= sa.B;
    const uint8_t* frame = (second ? next_obs : obs) +
                           (long long)sample_row(sa, second ? img0 - sa.B : img0) * Wsrc * Wsrc * C;
    if constexpr (SQK == 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) fw[c] = frame[(long long)p * C + c];
    } else {
#pragma unroll
      for (int r = 0; r < SQK; ++r) {
        const unsigned* w =
            reinterpret_cast<const unsigned*>(frame + ((long long)(y * SQK + r) * Wsrc + xq * SQK) * C);
#pragma unroll
        for (int q = 0; q < SEG / 4; ++q) fw[r * (SEG / 4) + q] = w[q];
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < RX; ++i) {
      const int e = (int)threadIdx.x + NT * i;
      xv[i] = e < gn * C * SD * SD ? x[(long long)img0 * C * SD * SD + e] : 0.f;
    }
  }
  const int c0w = ((threadIdx.x >> 6) % CT) * 16;
  WFrag<C, F, 0, SD> w0;
  WFrag<C, F, 1, SD> w1;
  WFrag<C, F, (NC > 2 ? 2 : 1), SD> w2;
  if constexpr (PRE) {
    w0.load(wp + E::F0, b0, c0w);
    w1.load(wp + E::F1, b1, c0w);
    if constexpr (NC > 2) w2.load(wp + E::F2, b2, c0w);
  }
  if constexpr (SQK > 0) {
    // each byte of the block rows into its channel's integer sum, then x
    int sum[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sum[c] = SQK == 1 ? (int)fw[c] : 0;
    if constexpr (SQK > 1) {
#pragma unroll
      for (int r = 0; r < SQK; ++r)
#pragma unroll
        for (int q = 0; q < SEG / 4; ++q) {
          const unsigned v = fw[r * (SEG / 4) + q];
#pragma unroll
          for (int b = 0; b < 4; ++b) sum[(4 * q + b) % C] += (int)((v >> (8 * b)) & 0xFFu);
        }
    }
    const float scale = (float)(255 * SQK * SQK);
    const int p = threadIdx.x;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float v = (float)sum[c] / scale - 0.5f;
      xout[((long long)img0 * C + c) * SD * SD + p] = v;
      lx[p * L0::PS + c] = (__bf16)v;
    }
  } else {
    // images NCHW -> [g][pixel][channel] bfloat16; absent images and padding channels zero
#pragma unroll
    for (int i = 0; i < RX; ++i) {
      const int e = (int)threadIdx.x + NT * i;
      if (e < G * C * SD * SD) {
        const int g = e / (C * SD * SD), r = e - g * C * SD * SD, c = r / (SD * SD), pix = r - c * SD * SD;
        lx[(g * SD * SD + pix) * L0::PS + c] = (__bf16)xv[i];
      }
    }
  }
  for (int e = threadIdx.x; e < G * SD * SD * (L0::CP - C); e += NT) {
    const int gp = e / (L0::CP - C), c = C + e - gp * (L0::CP - C);
    lx[gp * L0::PS + c] = (__bf16)0.f;
  }
  lds_barrier();
  conv_fwd_layer_b<G, C, F, 0, SD, true, false, NT, PRE>(lx, la0, wp + E::F0, b0, h0 + (long long)img0 * F * L0::P, gn,
                                                     w0);
  lds_barrier();
  if constexpr (NC > 2) {
    conv_fwd_layer_b<G, C, F, 1, SD, true, false, NT, PRE>(la0, la1, wp + E::F1, b1, h1 + (long long)img0 * F * L1::P,
                                                       gn, w1);
    lds_barrier();
    conv_fwd_layer_b<G, C, F, 2, SD, false, true, NT, PRE>(la1, nullptr, wp + E::F2, b2,
                                                       h2 + (long long)img0 * F * LB<C, F, 2, SD>::P, gn, w2,
                                                       reinterpret_cast<float*>(lx),
                                                       hh ? hh + (long long)img0 * F * LB<C, F, 2, SD>::P : nullptr);
  } else {
    conv_fwd_layer_b<G, C, F, 1, SD, false, true, NT, PRE>(la0, nullptr, wp + E::F1, b1,
                                                       h1 + (long long)img0 * F * L1::P, gn, w1,
                                                       reinterpret_cast<float*>(lx),
                                                       hh ? hh + (long long)img0 * F * L1::P : nullptr);
  }
}

// Weight gradient of layer l from D (bfloat16 [G][DS][DS][F + 8], zero border of
// 2) and the layer's input (bfloat16 [G][HI][HI][PS]): rows f, columns kc = c * 9
// + tap (the parameter order, so a tile's 16 columns are 16 consecutive floats of
// the partial gradient and its stores coalesce), contraction over the images'
// output pixels in 32-pixel chunks; each lane gathers its 8 pixels of a chunk
// through the position table (pixel -> offset in D, offset of its input patch
// origin), filled beforehand.
#ifndef SQ_ENC_QTAB
#define SQ_ENC_QTAB 1
#endif
#ifndef SQ_ENC_PREFETCH
#define SQ_ENC_PREFETCH 1
#endif
template <int G, int C, int F, int l, int SD, int NT>
__device__ __forceinline__ void fill_qtab(int2* qtab) {
  using Y = LB<C, F, l, SD>;
  constexpr int PSF = F + 8;
  constexpr int NPOS = G * Y::P, NQ = (NPOS + 31) / 32 * 32;
  for (int q = threadIdx.x; q < NQ; q += NT) {
    int2 e = make_int2(0, 0);   // pad entries: a zero border pixel of D, any finite input
    if (q < NPOS) {
      const int g = q / Y::P, p = q - g * Y::P, oy = p / Y::HO, ox = p - oy * Y::HO;
      e.x = ((g * Y::DS + oy + 2) * Y::DS + ox + 2) * PSF;
      e.y = ((g * Y::HI + oy * Y::S) * Y::HI + ox * Y::S) * Y::PS;
    }
    qtab[q] = e;
  }
}

template <int G, int C, int F, int l, int SD>
struct WTiles {
  using Y = LB<C, F, l, SD>;
  static constexpr int RT = F / 16, CT = (Y::K + 15) / 16, N = RT * CT;
};

template <int G, int C, int F, int l, int SD>
__device__ __forceinline__ void bwd_w_tile(int t, const __bf16* D, const __bf16* in, const int2* qtab,
                                           float* __restrict__ partW) {
  using Y = LB<C, F, l, SD>;
  using W = WTiles<G, C, F, l, SD>;
  constexpr int PSF = F + 8;
  constexpr int NPOS = G * Y::P, NQ = (NPOS + 31) / 32 * 32;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int rt = t / W::CT, ct = t - rt * W::CT;
  const int f0 = rt * 16, k0 = ct * 16;
  const int kc = min(k0 + li, Y::K - 1);
  const int c = kc / 9, tap = kc - 9 * c, ky = tap / 3, kx = tap - 3 * ky;
  const __bf16* ap = D + f0 + li;
  const __bf16* bp = in + (ky * Y::HI + kx) * Y::PS + c;
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NQ / 32; ++s) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      // output pixel q: its place in D and its input patch origin (pad pixels
      // read a zero border pixel of D against an arbitrary finite input)
      const int q = 32 * s + 8 * lq + e;
      int ox_d, ox_i;
      if constexpr (SQ_ENC_QTAB) {
        const int2 o = qtab[q];
        ox_d = o.x;
        ox_i = o.y;
      } else {
        const int qq = q < NPOS ? q : 0;
        const int g = qq / Y::P, p = qq - g * Y::P, oy = p / Y::HO, ox = p - oy * Y::HO;
        ox_d = q < NPOS ? ((g * Y::DS + oy + 2) * Y::DS + ox + 2) * PSF : 0;
        ox_i = ((g * Y::HI + oy * Y::S) * Y::HI + ox * Y::S) * Y::PS;
      }
      a[e] = ap[ox_d];
      b[e] = bp[ox_i];
    }
    acc = mma_b(a, b, acc);
  }
  const int kk = k0 + li;
  if (kk < Y::K) {
#pragma unroll
    for (int q = 0; q < 4; ++q) partW[(f0 + 4 * lq + q) * Y::K + kk] = acc[q];
  }
}

// Input gradient of layer l >= 1 from D_l (bfloat16): E[g][iy][ix][c] = sum over
// taps and f of D_l[g][iy - ky][ix - kx][f] W[f][c][ky][kx], masked by the layer's
// input (hin, FP32 [img][pixel][F]) > 0, into the interior of Dn (bfloat16,
// zero-bordered [G][HI + 4][HI + 4][F + 8]).  The masked FP32 values of each
// 16-row tile are also summed per channel into bpart[tile][c] (the bias gradient
// of layer l - 1, from unrounded values: lanes' rows in order, then the four
// lane groups as (0 + 1) + (2 + 3)).
template <int G, int C, int F, int l, int SD>
struct XTiles {
  using Y = LB<C, F, l, SD>;
  static constexpr int ROWS = G * Y::HI * Y::HI, RT = (ROWS + 15) / 16, CT = F / 16, N = RT * CT;
};

template <int G, int C, int F, int l, int SD>
__device__ __forceinline__ void bwd_x_tile(int t, const __bf16* D, const __bf16* __restrict__ wb,
                                           const float* __restrict__ hin, __bf16* Dn, float* bpart, int gn) {
  using Y = LB<C, F, l, SD>;
  using X = XTiles<G, C, F, l, SD>;
  static_assert(l >= 1, "input gradients are needed above the first layer only");
  constexpr int PSF = F + 8, DSN = Y::HI + 4;
  constexpr int TPM = 32 / F, NM = (9 + TPM - 1) / TPM;
  constexpr int ROWS = X::ROWS;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int rt = t / X::CT, ct = t - rt * X::CT;
  const int r0 = rt * 16, c0 = ct * 16;
  const int row = min(r0 + li, ROWS - 1);
  const int g = row / (Y::HI * Y::HI), pq = row - g * Y::HI * Y::HI, iy = pq / Y::HI, ix = pq - iy * Y::HI;
  const __bf16* ap = D + ((g * Y::DS + iy + 2) * Y::DS + ix + 2) * PSF;
  const __bf16* bp = wb + (c0 + li) * F;
  const int c = c0 + li;
  // the ReLU masks of this lane's four rows, requested before the contraction
  float hm[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = min(r0 + 4 * lq + q, ROWS - 1), gg = r / (Y::HI * Y::HI), pp = r - gg * Y::HI * Y::HI;
    hm[q] = gg < gn ? hin[((long long)gg * Y::HI * Y::HI + pp) * F + c] : 0.f;
  }
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mi = 0; mi < NM; ++mi) {
    int tap, off;
    chunk_tap<TPM>(mi, lq, tap, off);
    const int tc = tap < 9 ? tap : 8, ky = tc / 3, kx = tc - 3 * ky;
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap - (ky * Y::DS + kx) * PSF + off);
    bf16x8 b = *reinterpret_cast<const bf16x8*>(__builtin_assume_aligned(bp + tc * F * F + off, 16));
    if (tap > 8) b = bf16x8{};
    acc = mma_b(a, b, acc);
  }
  float sum = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + 4 * lq + q;
    if (r < ROWS) {
      const int gg = r / (Y::HI * Y::HI), pp = r - gg * Y::HI * Y::HI, yy = pp / Y::HI, xx = pp - yy * Y::HI;
      const float v = hm[q] > 0.f ? acc[q] : 0.f;
      Dn[((gg * DSN + yy + 2) * DSN + xx + 2) * PSF + c] = (__bf16)v;
      sum += v;
    }
  }
  sum += __shfl_xor(sum, 16);
  sum += __shfl_xor(sum, 32);
  if (lq == 0) bpart[rt * F + c] = sum;
}

// Both products of a layer l >= 1 share one pass over the waves (they read the
// same D_l and write different buffers): input-gradient tiles first (the longer
// ones), then weight-gradient tiles.  The position table must be filled.
template <int G, int C, int F, int l, int SD, int NT>
__device__ __forceinline__ void bwd_layer_b(const __bf16* D, const __bf16* in, const int2* qtab,
                                            float* __restrict__ partW, const __bf16* __restrict__ wb,
                                            const float* __restrict__ hin, __bf16* Dn, float* bpart, int gn) {
  using X = XTiles<G, C, F, l, SD>;
  using W = WTiles<G, C, F, l, SD>;
  const int wave = threadIdx.x >> 6;
  for (int t = wave; t < X::N + W::N; t += NT / 64) {
    if (t < X::N) bwd_x_tile<G, C, F, l, SD>(t, D, wb, hin, Dn, bpart, gn);
    else bwd_w_tile<G, C, F, l, SD>(t - X::N, D, in, qtab, partW);
  }
}

// every element e < N (stride NT) of a staging load, issued up front into registers
template <int N, int NT>
struct Prefetch {
  static constexpr int R = (N + NT - 1) / NT;
  float v[R > 0 ? R : 1];
  __device__ __forceinline__ void load(const float* __restrict__ src, int valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = (int)threadIdx.x + NT * i;
      v[i] = e < valid ? src[e] : 0.f;
    }
  }
};

template <int G, int C, int F, int NC, int SD, int NT>
__global__ __launch_bounds__(NT) void k_encoder_bwd_b(const float* __restrict__ x, int n,
                                                      const float* __restrict__ dfeat, const __bf16* __restrict__ wp,
                                                      const float* __restrict__ h0, const float* __restrict__ h1,
                                                      const float* __restrict__ h2, EncOffs off, long long enc_total,
                                                      float* __restrict__ part) {
  using L0 = LB<C, F, 0, SD>;
  using L1 = LB<C, F, 1, SD>;
  using L2 = LB<C, F, (NC > 2 ? 2 : 1), SD>;
  using LL = LB<C, F, NC - 1, SD>;
  using E = EncPrep<C, F, NC>;
  constexpr int PSF = F + 8;
  constexpr int SZ0 = G * L0::DS * L0::DS * PSF;                                  // D_0
  constexpr int SZ1 = G * L1::DS * L1::DS * PSF;                                  // D_1
  constexpr int SZ2 = NC > 2 ? G * L2::DS * L2::DS * PSF : 8;                     // D_2
  constexpr int R0 = SZ0 > SZ2 ? SZ0 : SZ2;   // D_2 first, D_0 last (never live together)
  constexpr int IN0 = G * SD * SD * L0::PS, IN1 = G * L1::HI * L1::HI * L1::PS;
  constexpr int RIN = IN0 > IN1 ? IN0 : IN1;
  constexpr int RTB = (G * L1::HI * L1::HI + 15) / 16;   // most 16-row tiles of an input gradient
  constexpr int TOPN = G * F * LL::P;                    // the top layer's upstream gradient elements
  constexpr int NH1 = NC > 2 ? G * L2::HI * L2::HI * F : 0, NH0 = G * L1::HI * L1::HI * F, NX = G * C * SD * SD;
  __shared__ __attribute__((aligned(16))) __bf16 r0[R0];
  __shared__ __attribute__((aligned(16))) __bf16 r1[SZ1];
  __shared__ __attribute__((aligned(16))) __bf16 rin[RIN];
  __shared__ float bpart[RTB * F > TOPN ? RTB * F : TOPN];
  __shared__ int2 qtab[(G * L0::P + 31) / 32 * 32];
  const int img0 = blockIdx.x * G;
  const int gn = n - img0 < G ? n - img0 : G;
  float* pp = part + (long long)blockIdx.x * enc_total;

  // every input the workgroup stages is requested now and lands in registers while
  // the layers above it are processed: the top layer's gradient and output, then
  // the inputs of layers 2, 1 and 0
  const float* hl = NC > 2 ? h2 : h1;
  Prefetch<TOPN, NT> pd, ph;
  pd.load(dfeat + (long long)img0 * F * LL::P, gn * F * LL::P);
  ph.load(hl + (long long)img0 * F * LL::P, gn * F * LL::P);
  Prefetch<NH1, NT> p1;
  Prefetch<NH0, NT> p0;
  Prefetch<NX, NT> px;
  auto load1 = [&] {
    if constexpr (NC > 2) p1.load(h1 + (long long)img0 * L2::HI * L2::HI * F, gn * L2::HI * L2::HI * F);
  };
  auto load0 = [&] { p0.load(h0 + (long long)img0 * L1::HI * L1::HI * F, gn * L1::HI * L1::HI * F); };
  auto loadx = [&] { px.load(x + (long long)img0 * C * SD * SD, gn * C * SD * SD); };
  if constexpr (SQ_ENC_PREFETCH) {
    load1();
    load0();
    loadx();
  }

  // D_{NC-1}: zero, then the upstream gradient (NCHW) masked by the output > 0 into
  // the interior; its bias gradient sums the same FP32 values, thread f in (g, p) order
  __bf16* Dl = NC > 2 ? r0 : r1;
  for (int e = threadIdx.x; e < (NC > 2 ? SZ2 : SZ1); e += NT) Dl[e] = (__bf16)0.f;
  lds_barrier();
#pragma unroll
  for (int i = 0; i < Prefetch<TOPN, NT>::R; ++i) {
    const int e = (int)threadIdx.x + NT * i;
    if (e < TOPN) {
      const int g = e / (F * LL::P), r = e - g * F * LL::P, f = r / LL::P, p = r - f * LL::P;
      const int oy = p / LL::HO, ox = p - oy * LL::HO;
      const float v = ph.v[i] > 0.f ? pd.v[i] : 0.f;
      Dl[((g * LL::DS + oy + 2) * LL::DS + ox + 2) * PSF + f] = (__bf16)v;
      bpart[e] = v;
    }
  }
  lds_barrier();
  if (threadIdx.x < F) {
    const int f = threadIdx.x;
    float sb = 0.f;
    for (int g = 0; g < G; ++g)
      for (int p = 0; p < LL::P; ++p) sb += bpart[(g * F + f) * LL::P + p];
    pp[off.b[NC - 1] + f] = sb;
  }
  if constexpr (NC > 2) {
    // layer 2: input h1 ([img][pixel][F] -> [g][pixel][PS]); D_2 in r0, D_1 -> r1
    if constexpr (!SQ_ENC_PREFETCH) load1();
#pragma unroll
    for (int i = 0; i < Prefetch<NH1, NT>::R; ++i) {
      const int e = (int)threadIdx.x + NT * i;
      if (e < NH1) rin[(e / F) * L2::PS + e % F] = (__bf16)p1.v[i];
    }
    for (int e = threadIdx.x; e < SZ1; e += NT) r1[e] = (__bf16)0.f;
    fill_qtab<G, C, F, 2, SD, NT>(qtab);
    lds_barrier();
    bwd_layer_b<G, C, F, 2, SD, NT>(r0, rin, qtab, pp + off.W[2], wp + E::B2,
                                h1 + (long long)img0 * L2::HI * L2::HI * F, r1, bpart, gn);
    lds_barrier();
    if (threadIdx.x < F) {
      float sb = 0.f;
      for (int t = 0; t < (G * L2::HI * L2::HI + 15) / 16; ++t) sb += bpart[t * F + threadIdx.x];
      pp[off.b[1] + threadIdx.x] = sb;
    }
  }
  // layer 1: input h0; D_1 in r1, D_0 -> r0
  if constexpr (!SQ_ENC_PREFETCH) load0();
#pragma unroll
  for (int i = 0; i < Prefetch<NH0, NT>::R; ++i) {
    const int e = (int)threadIdx.x + NT * i;
    if (e < NH0) rin[(e / F) * L1::PS + e % F] = (__bf16)p0.v[i];
  }
  for (int e = threadIdx.x; e < SZ0; e += NT) r0[e] = (__bf16)0.f;
  fill_qtab<G, C, F, 1, SD, NT>(qtab);
  lds_barrier();
  bwd_layer_b<G, C, F, 1, SD, NT>(r1, rin, qtab, pp + off.W[1], wp + E::B1, h0 + (long long)img0 * L1::HI * L1::HI * F,
                              r0, bpart, gn);
  lds_barrier();
  if (threadIdx.x < F) {
    float sb = 0.f;
    for (int t = 0; t < (G * L1::HI * L1::HI + 15) / 16; ++t) sb += bpart[t * F + threadIdx.x];
    pp[off.b[0] + threadIdx.x] = sb;
  }
  // layer 0: input x (NCHW -> [g][pixel][channel], padding channels zero); D_0 in r0
  if constexpr (!SQ_ENC_PREFETCH) loadx();
#pragma unroll
  for (int i = 0; i < Prefetch<NX, NT>::R; ++i) {
    const int e = (int)threadIdx.x + NT * i;
    if (e < NX) {
      const int g = e / (C * SD * SD), r = e - g * C * SD * SD, c = r / (SD * SD), pix = r - c * SD * SD;
      rin[(g * SD * SD + pix) * L0::PS + c] = (__bf16)px.v[i];
    }
  }
  for (int e = threadIdx.x; e < G * SD * SD * (L0::CP - C); e += NT) {
    const int gp = e / (L0::CP - C), c = C + e - gp * (L0::CP - C);
    rin[gp * L0::PS + c] = (__bf16)0.f;
  }
  fill_qtab<G, C, F, 0, SD, NT>(qtab);
  lds_barrier();
  for (int t = threadIdx.x >> 6; t < WTiles<G, C, F, 0, SD>::N; t += NT / 64)
    bwd_w_tile<G, C, F, 0, SD>(t, r0, rin, qtab, pp + off.W[0]);
}

// ---------------------------------------------------------------- launchers
constexpr int kEncFwdG = 2, kEncFwdThreads = 512;
constexpr int kEncBwdG = 2, kEncBwdThreads = 512;
// measured on the full network, B = 512 (forward / backward per update): one image and
// 256 threads per forward workgroup 14.5 us (two images, 512 threads: 14.9; four, 512:
// 18.1); 1024 threads per backward workgroup 27.2 us (512: 31.5; 256: 41.4)
#ifndef SQ_ENC_FWD_G
#define SQ_ENC_FWD_G 1
#endif
#ifndef SQ_ENC_FWD_T
#define SQ_ENC_FWD_T 256
#endif
#ifndef SQ_ENC_BWD_T
#define SQ_ENC_BWD_T 1024
#endif
// bfloat16 form (the backward keeps kEncBwdG images per workgroup: the partial-gradient rows follow it)
constexpr int kEncFwdGb = SQ_ENC_FWD_G, kEncFwdThreadsb = SQ_ENC_FWD_T;
constexpr int kEncBwdThreadsb = SQ_ENC_BWD_T;

template <int C, int F, int NC>
static int prep_t(const float* const* W, float* wp, int bf16, hipStream_t st) {
  EncW w{{W[0], W[1], NC > 2 ? W[2] : W[1]}};
  const int tot = EncPrep<C, F, NC>::TOTAL;
  k_enc_prep<C, F, NC><<<cdiv(tot, 256), 256, 0, st>>>(w, wp, bf16);
  return launch_status("encoder_prep");
}

// images per backward workgroup (the partial-gradient rows follow it): two on 16 x 16
// inputs, one on 32 x 32 (whose LDS holds one image's activations and gradients)
constexpr int enc_bwd_g(int side) { return side == 16 ? kEncBwdG : 1; }

template <bool BF16, int C, int F, int NC, int SD>
static int enc_fwd_t(const float* x, int n, const float* wp, const float* const* b, float* const* h, uint16_t* hh,
                     hipStream_t st) {
  if constexpr (BF16) {
    const int nwg = cdiv(n, kEncFwdGb);
    k_encoder_fwd_b<kEncFwdGb, C, F, NC, SD, kEncFwdThreadsb><<<nwg, kEncFwdThreadsb, 0, st>>>(
        x, n, reinterpret_cast<const __bf16*>(wp), b[0], b[1], NC > 2 ? b[2] : b[1], h[0], h[1],
        NC > 2 ? h[2] : h[1], hh, nullptr, nullptr, SampleArgs{}, 0, nullptr);
  } else {
    static_assert(SD == 16, "the FP32 fused encoder is built for 16 x 16 inputs");
    const int nwg = cdiv(n, kEncFwdG);
    k_encoder_fwd<false, kEncFwdG, C, F, NC, kEncFwdThreads><<<nwg, kEncFwdThreads, 0, st>>>(
        x, n, wp, b[0], b[1], NC > 2 ? b[2] : b[1], h[0], h[1], NC > 2 ? h[2] : h[1]);
  }
  return launch_status("encoder_fwd");
}

int encoder_fused_part_rows(int n, int side) { return cdiv(n, enc_bwd_g(side)); }

template <int C, int F, int NC>
static void prep_map_t(const long long* W, EncPrepMap* m) {
  using E = EncPrep<C, F, NC>;
  m->n = NC;
  m->F = F;
  const long long fb[3] = {E::F0, E::F1, E::F2}, bb[3] = {-1, E::B1, E::B2};
  const int cp[3] = {LG<C, F, 0>::CP, LG<C, F, 1>::CP, LG<C, F, 2>::CP};
  m->lo = W[0];
  m->hi = W[0];
  for (int l = 0; l < NC; ++l) {
    m->W[l] = W[l];
    m->cin[l] = l == 0 ? C : F;
    m->cp[l] = cp[l];
    m->fb[l] = fb[l];
    m->bb[l] = bb[l];
    const long long end = W[l] + (long long)F * m->cin[l] * 9;
    m->hi = end > m->hi ? end : m->hi;
  }
}

bool encoder_fused_prep_map(int C, int F, int n_conv, int side, const long long* W, float* wp, int bf16,
                            EncPrepMap* m) {
  if (!encoder_fused_ok(C, F, n_conv, side, bf16) || !wp) return false;
  *m = EncPrepMap{};
  if (C == 9 && F == 32 && n_conv == 3) prep_map_t<9, 32, 3>(W, m);
  else prep_map_t<3, 16, 2>(W, m);
  m->wp = wp;
  m->bf16 = bf16;
  return true;
}

template <bool BF16, int C, int F, int NC, int SD>
static int enc_bwd_t(const float* x, int n, const float* dfeat, const float* wp, const float* const* h,
                     const long long* Woff, const long long* boff, long long total, float* part, float* grad,
                     hipStream_t st) {
  constexpr int GB = enc_bwd_g(SD);
  const int nwg = cdiv(n, GB);
  EncOffs off{};
  for (int i = 0; i < NC; ++i) {
    off.W[i] = Woff[i];
    off.b[i] = boff[i];
  }
  if constexpr (BF16) {
    k_encoder_bwd_b<GB, C, F, NC, SD, kEncBwdThreadsb><<<nwg, kEncBwdThreadsb, 0, st>>>(
        x, n, dfeat, reinterpret_cast<const __bf16*>(wp), h[0], h[1], NC > 2 ? h[2] : h[1], off, total, part);
  } else {
    static_assert(SD == 16, "the FP32 fused encoder is built for 16 x 16 inputs");
    k_encoder_bwd<false, kEncBwdG, C, F, NC, kEncBwdThreads><<<nwg, kEncBwdThreads, 0, st>>>(
        x, n, dfeat, wp, h[0], h[1], NC > 2 ? h[2] : h[1], off, total, part);
  }
  SQ_TRY(launch_status("encoder_bwd"));
  if (!grad) return SQ_OK;   // the caller sums the partials (an optimiser segment)
  k_enc_reduce<<<(int)cdiv(total, 256), 256, 0, st>>>(part, nwg, total, grad);
  return launch_status("encoder_reduce");
}

bool encoder_fused_ok(int C, int F, int n_conv, int side, int bf16) {
  if (side == 16) return (C == 9 && F == 32 && n_conv == 3) || (C == 3 && F == 16 && n_conv == 2);
  return side == 32 && bf16 && C == 9 && F == 32 && n_conv == 3;   // bfloat16 form only
}

size_t encoder_fused_part_floats(int n, long long enc_total, int side) {
  return (size_t)encoder_fused_part_rows(n, side) * enc_total;
}

size_t encoder_fused_prep_floats(int C, int F, int n_conv) {
  if (C == 9 && F == 32 && n_conv == 3) return EncPrep<9, 32, 3>::TOTAL;
  return EncPrep<3, 16, 2>::TOTAL;
}

int encoder_fused_prep(int bf16, int C, int F, int n_conv, const float* const* W, float* wp, hipStream_t st) {
  if (C == 9 && F == 32 && n_conv == 3) return prep_t<9, 32, 3>(W, wp, bf16, st);
  return prep_t<3, 16, 2>(W, wp, bf16, st);
}

int encoder_fused_fwd(int bf16, int C, int F, int n_conv, int side, const float* x, int n, const float* wp,
                      const float* const* b, float* const* h, hipStream_t st, uint16_t* hh) {
  if (n <= 0) return SQ_OK;
  if (hh && !bf16) {
    set_error("encoder_fused_fwd: the feature's bfloat16 copy is written by the bfloat16 form only");
    return SQ_EINVAL;
  }
  if (side == 32) return enc_fwd_t<true, 9, 32, 3, 32>(x, n, wp, b, h, hh, st);
  if (C == 9 && F == 32 && n_conv == 3)
    return bf16 ? enc_fwd_t<true, 9, 32, 3, 16>(x, n, wp, b, h, hh, st)
                : enc_fwd_t<false, 9, 32, 3, 16>(x, n, wp, b, h, nullptr, st);
  return bf16 ? enc_fwd_t<true, 3, 16, 2, 16>(x, n, wp, b, h, hh, st)
              : enc_fwd_t<false, 3, 16, 2, 16>(x, n, wp, b, h, nullptr, st);
}

int encoder_fused_fwd_squint(const SampleArgs& sa, const uint8_t* obs, const uint8_t* next_obs, int H, int W, int C,
                             int F, int n_conv, int k, float* x, const float* wp, const float* const* b,
                             float* const* h, uint16_t* hh, hipStream_t st) {
  const int n = 2 * sa.B;
  if (n <= 0) return SQ_OK;
  // the headline geometry: 64 x 64 x 9 frames squinted 4x (or their 16 x 16 block means stored in a
  // ring, k = 1) into the 16 x 16 encoder, one image per 256-thread workgroup (a thread per output pixel)
  if (!(C == 9 && F == 32 && n_conv == 3 && kEncFwdGb == 1 && kEncFwdThreadsb == 256)) return kNotApplicable;
  const bool raw = k == 4 && H == 64 && W == 64 && (uintptr_t)obs % 4 == 0 && (uintptr_t)next_obs % 4 == 0;
  const bool stored = k == 1 && H == 16 && W == 16;
  if (!raw && !stored) return kNotApplicable;
  const int lead = (int)((sample_items(sa.B, sa.A, sa.S) + kEncFwdThreadsb - 1) / kEncFwdThreadsb);
  const __bf16* wb = reinterpret_cast<const __bf16*>(wp);
  if (raw)
    k_encoder_fwd_b<1, 9, 32, 3, 16, 256, 4><<<lead + n, 256, 0, st>>>(nullptr, n, wb, b[0], b[1], b[2], h[0], h[1],
                                                                       h[2], hh, obs, next_obs, sa, lead, x);
  else
    k_encoder_fwd_b<1, 9, 32, 3, 16, 256, 1><<<lead + n, 256, 0, st>>>(nullptr, n, wb, b[0], b[1], b[2], h[0], h[1],
                                                                       h[2], hh, obs, next_obs, sa, lead, x);
  return launch_status("encoder_fwd_squint");
}

int encoder_fused_bwd(int bf16, int C, int F, int n_conv, int side, const float* x, int n, const float* dfeat,
                      const float* wp, const float* const* h, const long long* Woff, const long long* boff,
                      long long total, float* part, float* grad, hipStream_t st) {
  if (n <= 0) return SQ_OK;
  if (side == 32) return enc_bwd_t<true, 9, 32, 3, 32>(x, n, dfeat, wp, h, Woff, boff, total, part, grad, st);
  if (C == 9 && F == 32 && n_conv == 3)
    return bf16 ? enc_bwd_t<true, 9, 32, 3, 16>(x, n, dfeat, wp, h, Woff, boff, total, part, grad, st)
                : enc_bwd_t<false, 9, 32, 3, 16>(x, n, dfeat, wp, h, Woff, boff, total, part, grad, st);
  return bf16 ? enc_bwd_t<true, 3, 16, 2, 16>(x, n, dfeat, wp, h, Woff, boff, total, part, grad, st)
              : enc_bwd_t<false, 3, 16, 2, 16>(x, n, dfeat, wp, h, Woff, boff, total, part, grad, st);
}

}  // namespace sq
