// Dense products on the matrix cores (MFMA) of gfx950.
//
// One kernel template covers every contraction of the update: the linear layers
// (forward, input gradient, weight gradient) and the 3x3 convolutions as implicit
// GEMMs.  Operands are read through "fetchers" that map a logical element
// (row, k) to memory, so transposes, concatenated inputs, im2col patches and the
// ReLU mask of a convolution's gradient are all folded into the tile loads.
//
// Tiling: a 256-thread workgroup owns a 32 x 32 output tile.  Each K step stages
// a 32 x BK slice of both operands in LDS (converted to the compute type: FP32,
// or bfloat16 rounded to nearest even), and the four waves each contract a
// quarter of the slice (16 k for FP32 with v_mfma_f32_16x16x4_f32, 32 k for
// bfloat16 with v_mfma_f32_16x16x32_bf16), accumulating in FP32 registers.  At
// the end the four partial tiles are summed through LDS in a fixed order, so the
// result is independent of scheduling.  Long reductions (conv weight gradients)
// are split over K across workgroups into a scratch buffer and summed in order
// by a second kernel.
//
// Workgroup order: consecutive workgroups go to the eight XCDs in turn, each
// with its own L2, so the linear workgroup id is remapped (when the tile count
// is a multiple of 8) to give every XCD a contiguous run of tiles, ordered in
// groups of 8 row tiles -- about an 8 x 8 block of tiles per XCD, which reads
// half of each operand of its batch instead of all of one operand.
#include "../common.h"
#include "bf16.h"
#include "tgauss.h"

#include <algorithm>
#include <type_traits>

namespace sq {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kTile = 32;

template <bool BF16> struct Cfg;
template <> struct Cfg<false> {
  using T = float;
  static constexpr int KW = 16;   // k per wave per step
  static constexpr int PAD = 1;
};
template <> struct Cfg<true> {
  using T = uint16_t;             // bfloat16 bits
  static constexpr int KW = 32;
  static constexpr int PAD = 8;   // keeps 16-byte alignment of every 8-element group
};

__device__ __forceinline__ float to_t(float v, float*) { return v; }
__device__ __forceinline__ uint16_t to_t(float v, uint16_t*) { return bf16_bits(v); }

// ---------------------------------------------------------------- fetchers
// KFAST: consecutive k are adjacent in memory (coalesce along k), else along rows.
template <bool KF> struct FMat {
  const float* p; long long lr, lk, sz;
  static constexpr bool KFAST = KF;
  __device__ __forceinline__ float get(int z, int r, int k) const { return p[z * sz + r * lr + k * lk]; }
};

// Convolution geometry: input side H, output side HO, stride S.  The encoder's
// shapes are compile-time constants (so the index divisions become multiplies);
// Geo<0, 0, 0> carries them at run time for any other shape.
template <int H_, int HO_, int S_> struct Geo {
  int h, ho, s;
  __device__ __forceinline__ int H() const { return H_ ? H_ : h; }
  __device__ __forceinline__ int HO() const { return HO_ ? HO_ : ho; }
  __device__ __forceinline__ int S() const { return S_ ? S_ : s; }
};

// im2col of an NCHW input: row = (n, oy, ox), k = (c, ky, kx)
template <class G> struct FConvPatch {
  const float* x; int Cin; G g;
  static constexpr bool KFAST = false;
  __device__ __forceinline__ float get(int, int r, int k) const {
    const int Ho = g.HO(), H = g.H(), HoWo = Ho * Ho;
    const int n = r / HoWo, p = r - n * HoWo, oy = p / Ho, ox = p - oy * Ho;
    const int c = k / 9, t = k - 9 * c, ky = t / 3, kx = t - 3 * ky;
    return x[(((long long)n * Cin + c) * H + oy * g.S() + ky) * H + ox * g.S() + kx];
  }
};
// the same patch matrix transposed: row = (c, ky, kx), k = (n, oy, ox)
template <class G> struct FConvPatchT {
  FConvPatch<G> f;
  static constexpr bool KFAST = true;
  __device__ __forceinline__ float get(int z, int r, int k) const { return f.get(z, k, r); }
};
// gradient at a conv's pre-activation, transposed: row = f, k = (n, p); the
// upstream gradient is masked by the conv's ReLU output
template <class G> struct FConvGradT {
  const float* dout; const float* out; int F; G g;
  static constexpr bool KFAST = true;
  __device__ __forceinline__ float get(int, int r, int k) const {
    const int HoWo = g.HO() * g.HO();
    const int n = k / HoWo, p = k - n * HoWo;
    const long long i = ((long long)n * F + r) * HoWo + p;
    return out[i] > 0.f ? dout[i] : 0.f;
  }
};
// input gradient of a stride-1 conv: row = (n, iy, ix), k = (f, ky, kx)
template <class G> struct FConvDxA {
  const float* dout; const float* out; int F; G g;
  static constexpr bool KFAST = false;
  __device__ __forceinline__ float get(int, int r, int k) const {
    const int Hin = g.H(), Ho = g.HO(), HW = Hin * Hin;
    const int n = r / HW, q = r - n * HW, iy = q / Hin, ix = q - iy * Hin;
    const int f = k / 9, t = k - 9 * f, ky = t / 3, kx = t - 3 * ky;
    const int oy = iy - ky, ox = ix - kx;
    if (oy < 0 || oy >= Ho || ox < 0 || ox >= Ho) return 0.f;
    const long long i = (((long long)n * F + f) * Ho + oy) * Ho + ox;
    return out[i] > 0.f ? dout[i] : 0.f;
  }
};
// conv weights seen as B(c, (f, ky, kx)) = W[f][c][ky][kx]
struct FConvDxB {
  const float* W; int Cin;
  static constexpr bool KFAST = true;
  __device__ __forceinline__ float get(int, int r, int k) const {
    const int f = k / 9, t = k - 9 * f;
    return W[((long long)f * Cin + r) * 9 + t];
  }
};

// ---------------------------------------------------------------- stores
struct StMat {
  float* p; long long ld, sz; const float* bias; long long bias_sz; int acc, relu;
  const float* bias_alt = nullptr; int bias_zalt = kNoAlt;
  static constexpr bool ROW_FAST = false;
  static constexpr bool ROWS = false;   // element stores (put), not a tile epilogue
  __device__ void rows(int, int, const float*, int, float*) const {}
  __device__ __forceinline__ void put(int z, int r, int c, float v) const {
    const long long i = z * sz + (long long)r * ld + c;
    if (bias) v += z < bias_zalt ? bias[z * bias_sz + c] : bias_alt[(z - bias_zalt) * bias_sz + c];
    if (acc) v += p[i];
    if (relu) v = fmaxf(v, 0.f);
    p[i] = v;
  }
};
// Tile epilogue of the policy head (N = 2A <= 32, one column tile): every thread
// takes one (row, dimension) of the tile: the head values (+ bias) go through the
// tanh-Gaussian sample (eps given) or the mean action tanh(mu) (eps null); log pi
// sums each row's dimension terms in d order; head itself is stored when wanted.
// v: the tile's sums [32][ld]; tmp: >= 32 * 32 floats of LDS.  All threads call.
struct StTanhGauss {
  const float* bias; const float* eps; float lo, hi; float* action; float* logp; float* save; float* head; int A;
  float* xact; long long ld_xact; int xact_row0;   // second copy of the actions of rows >= xact_row0 (nullable)
  uint16_t* xact_h;                                 // bfloat16 copy of xact's buffer (nullable)
  static constexpr bool ROW_FAST = false;
  static constexpr bool ROWS = true;
  __device__ void put(int, int, int, float) const {}
  __device__ void rows(int r0, int nr, const float* v, int ld, float* tmp) const {
    const int t = threadIdx.x, N = 2 * A;
    for (int e = t; e < nr * N; e += blockDim.x) {
      const int r = e / N, c = e - r * N;
      if (head) head[(long long)(r0 + r) * N + c] = v[r * ld + c] + (bias ? bias[c] : 0.f);
    }
    for (int e = t; e < nr * A; e += blockDim.x) {
      const int r = e / A, d = e - r * A;
      const long long row = r0 + r;
      const float mu = v[r * ld + d] + (bias ? bias[d] : 0.f);
      float act;
      if (eps) {
        const float us = v[r * ld + A + d] + (bias ? bias[A + d] : 0.f);
        tmp[r * 32 + d] = tanh_gauss_dim(mu, us, eps[row * A + d], A, d, lo, hi, action + row * A, save + row * 3 * A);
        act = save[row * 3 * A + 2 * A + d];
      } else {
        act = tanhf(mu);
        action[row * A + d] = act;
      }
      if (xact && row >= xact_row0) {
        xact[(row - xact_row0) * ld_xact + d] = act;
        if (xact_h) xact_h[(row - xact_row0) * ld_xact + d] = bf16_bits(act);
      }
    }
    if (!eps || !logp) return;
    __syncthreads();
    if (t < nr) {
      float lp = 0.f;
      for (int d = 0; d < A; ++d) lp += tmp[t * 32 + d];
      logp[r0 + t] = lp;
    }
  }
};
// The policy head's backward on a tile of da rows (v: [32][ld], columns < A), the
// same arithmetic as the standalone kernel: du = da (1 - a^2) + dlogp 2a,
// d u_s = (du sigma eps - dlogp) (hi - lo) / 2 (1 - tanh^2 u_s); with part, the
// tile's column sums of dhead (rows in order) go to part[r0 / 32][2A].
struct StTgBwd {
  const float* save; const float* eps; const float* dlogp_vec; const float* dlogp_scalar; float scale, lo, hi;
  float* dhead; float* part; int A;
  int ldh;             // dhead's row stride
  uint16_t* dhead_h;   // its bfloat16 copy (nullable)
  int off;             // da starts at column off of the tile
  static constexpr bool ROW_FAST = false;
  static constexpr bool ROWS = true;
  __device__ void put(int, int, int, float) const {}
  __device__ void rows(int r0, int nr, const float* v, int ld, float* tmp) const {
    const int t = threadIdx.x, N = 2 * A;
    for (int e = t; e < nr * A; e += blockDim.x) {
      const int r = e / A, d = e - r * A;
      const long long row = r0 + r;
      float dl = 0.f;
      if (dlogp_vec) dl += dlogp_vec[row];
      if (dlogp_scalar) dl += *dlogp_scalar * scale;
      const float tus = save[row * 3 * A + d];
      const float sd = save[row * 3 * A + A + d];
      const float a = save[row * 3 * A + 2 * A + d];
      const float du = v[r * ld + off + d] * (1.f - a * a) + dl * 2.f * a;
      const float dls = du * sd * eps[row * A + d] - dl;
      const float dls_out = dls * 0.5f * (hi - lo) * (1.f - tus * tus);
      dhead[row * ldh + d] = du;
      dhead[row * ldh + A + d] = dls_out;
      if (dhead_h) {
        dhead_h[row * ldh + d] = bf16_bits(du);
        dhead_h[row * ldh + A + d] = bf16_bits(dls_out);
      }
      tmp[r * N + d] = du;
      tmp[r * N + A + d] = dls_out;
    }
    if (!part) return;
    __syncthreads();
    for (int j = t; j < N; j += blockDim.x) {
      float sum = 0.f;
      for (int r = 0; r < nr; ++r) sum += tmp[r * N + j];
      part[(long long)(r0 / kTile) * N + j] = sum;
    }
  }
};
// C((n, p), c) -> out[n][c][p] (NCHW), optional bias + ReLU
struct StConv {
  float* out; int Cout, HW; const float* bias; int relu;
  static constexpr bool ROW_FAST = true;
  __device__ __forceinline__ void put(int, int r, int c, float v) const {
    const int n = r / HW, p = r - n * HW;
    if (bias) v += bias[c];
    if (relu) v = fmaxf(v, 0.f);
    out[((long long)n * Cout + c) * HW + p] = v;
  }
};
// split-K partial: part[(z * splits + s) * M * N + r * N + c]
struct StPart {
  float* part; int M, N, splits;
  __device__ __forceinline__ void put(int z, int s, int r, int c, float v) const {
    part[(((long long)z * splits + s) * M + r) * N + c] = v;
  }
};

// ---------------------------------------------------------------- kernel
// Global -> register staging of one 32 x BK operand slice.  Each thread owns
// EL = 32 * BK / 256 elements at fixed positions; all EL loads are issued back
// to back (bounds give zero), so their latencies overlap, and the next slice is
// fetched while the current one is being multiplied.
template <class F, int BK, int EL>
__device__ __forceinline__ void fetch(const F& f, float (&r)[EL], int z, int row0, int rows, int k0, int kend) {
#pragma unroll
  for (int i = 0; i < EL; ++i) {
    const int e = (int)threadIdx.x + kThreads * i;
    int rr, kk;
    if constexpr (F::KFAST) { rr = e / BK; kk = e - rr * BK; } else { kk = e / kTile; rr = e - kk * kTile; }
    const int gr = row0 + rr, gk = k0 + kk;
    r[i] = (gr < rows && gk < kend) ? f.get(z, gr, gk) : 0.f;
  }
}

template <class F, int BK, int LD, int EL, class T>
__device__ __forceinline__ void stage(const float (&r)[EL], T* tile) {
#pragma unroll
  for (int i = 0; i < EL; ++i) {
    const int e = (int)threadIdx.x + kThreads * i;
    int rr, kk;
    if constexpr (F::KFAST) { rr = e / BK; kk = e - rr * BK; } else { kk = e / kTile; rr = e - kk * kTile; }
    tile[rr * LD + kk] = to_t(r[i], (T*)nullptr);
  }
}

// Main loop: the operand slices of the next STAGES K-steps are in flight in
// registers at any time (the loop is unrolled by STAGES so every register slot
// is a compile-time index), so the global-load latency is paid about once per
// STAGES steps instead of once per step.
template <bool BF16, int LD>
__device__ __forceinline__ void mma_step(const typename Cfg<BF16>::T* As, const typename Cfg<BF16>::T* Bs,
                                         v4f (&acc)[2][2], int wave, int li, int lq) {
  using C = Cfg<BF16>;
  if constexpr (!BF16) {
#pragma unroll
    for (int kk = 0; kk < C::KW; kk += 4) {
      const int kq = wave * C::KW + kk + lq;
      const float a0 = As[li * LD + kq], a1 = As[(16 + li) * LD + kq];
      const float b0 = Bs[li * LD + kq], b1 = Bs[(16 + li) * LD + kq];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  } else {
    const int kq = wave * 32 + 8 * lq;
    const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&As[li * LD + kq]);
    const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&As[(16 + li) * LD + kq]);
    const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&Bs[li * LD + kq]);
    const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&Bs[(16 + li) * LD + kq]);
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
  }
}

template <bool BF16, class FA, class FB, class ST, bool SPLIT>
__global__ __launch_bounds__(kThreads) void k_gemm(FA fa, FB fb, ST st, StPart sp, int M, int N, int K,
                                                   int kchunk) {
  using C = Cfg<BF16>;
  using T = typename C::T;
  constexpr int BK = 4 * C::KW;
  constexpr int LD = BK + C::PAD;
  constexpr int EL = kTile * BK / kThreads;
#ifdef SQ_GEMM_STAGES
  constexpr int STAGES = SQ_GEMM_STAGES;
#else
  constexpr int STAGES = 2;
#endif
  constexpr int TILE_BYTES = 2 * kTile * LD * (int)sizeof(T);
  constexpr int RED_BYTES = 4 * kTile * (kTile + 1) * 4;
  constexpr int LDS_BYTES = TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES;
  __shared__ __attribute__((aligned(16))) char lds[LDS_BYTES];
  T* As = reinterpret_cast<T*>(lds);
  T* Bs = As + kTile * LD;

  const int z = blockIdx.z / (SPLIT ? sp.splits : 1);
  const int split = SPLIT ? blockIdx.z % sp.splits : 0;
  const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * kTile;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;

  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  float ra[STAGES][EL], rb[STAGES][EL];
#pragma unroll
  for (int s = 0; s < STAGES; ++s) {
    if (s < nk) {
      fetch<FA, BK, EL>(fa, ra[s], z, m0, M, kbeg + s * BK, kend);
      fetch<FB, BK, EL>(fb, rb[s], z, n0, N, kbeg + s * BK, kend);
    }
  }
  for (int kt = 0; kt < nk; kt += STAGES) {
#pragma unroll
    for (int s = 0; s < STAGES; ++s) {
      const int t = kt + s;
      if (t < nk) {
        stage<FA, BK, LD, EL>(ra[s], As);
        stage<FB, BK, LD, EL>(rb[s], Bs);
        __syncthreads();
        if (t + STAGES < nk) {
          fetch<FA, BK, EL>(fa, ra[s], z, m0, M, kbeg + (t + STAGES) * BK, kend);
          fetch<FB, BK, EL>(fb, rb[s], z, n0, N, kbeg + (t + STAGES) * BK, kend);
        }
        mma_step<BF16, LD>(As, Bs, acc, wave, li, lq);
        __syncthreads();
      }
    }
  }

  // fixed-order sum of the four waves' partial tiles
  float* red = reinterpret_cast<float*>(lds);
  constexpr int RLD = kTile + 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        red[(wave * kTile + i * 16 + 4 * lq + q) * RLD + j * 16 + li] = acc[i][j][q];
  __syncthreads();
  for (int e = threadIdx.x; e < kTile * kTile; e += kThreads) {
    int r, c;
    if constexpr (!SPLIT && ST::ROW_FAST) { c = e / kTile; r = e - c * kTile; } else { r = e / kTile; c = e - r * kTile; }
    const float v = ((red[(0 * kTile + r) * RLD + c] + red[(1 * kTile + r) * RLD + c]) +
                     red[(2 * kTile + r) * RLD + c]) + red[(3 * kTile + r) * RLD + c];
    const int gr = m0 + r, gc = n0 + c;
    if (gr < M && gc < N) {
      if constexpr (SPLIT) sp.put(z, split, gr, gc, v); else st.put(z, gr, gc, v);
    }
  }
}

// ---------------------------------------------------------------- plain-matrix kernel
// For plain strided operands (every linear layer).  Each wave contracts its
// quarter of the workgroup's K range for the whole 32 x 32 tile, in chunks of
// 32 k; lane (li, lq) feeds rows li and 16 + li at k = 8*lq .. 8*lq + 7 of a
// chunk to the matrix cores (one v_mfma_f32_16x16x32_bf16, or eight
// v_mfma_f32_16x16x4_f32 steps with step e taking k = 8*lq + e).
//
// Operand loads.  An operand whose rows are k-contiguous and 16-byte aligned is
// read row-coalesced -- eight consecutive lanes cover the 128 bytes of one row's
// chunk -- and rearranged into the fragment order through a small LDS tile that
// belongs to the wave alone (no workgroup barrier; the wave waits for its own
// LDS writes before reading back).  Reading the fragment order straight from
// memory would send each lane to a different row and costs the load unit several
// times more.  Other operands (k strided, rows contiguous) are read in fragment
// order directly, which is already coalesced across li.
//
// Chunks are fetched in groups of two, the next group in flight while the
// current one is multiplied.  The four partial tiles are summed through LDS in a
// fixed order at the end.  bfloat16 operands are rounded to nearest even
// (v_cvt_pk_bf16_f32) on the way to LDS or to the fragment.
struct RMat {
  const float* p; long long lr, lk, sz;
  const float* alt; int zalt, zdiv;   // batch groups, as MatArg
  const float* kp; int kalt;          // k >= kalt read from kp at k - kalt, as MatArg
  __device__ __forceinline__ const float* batch(int z) const {
    const int zi = z / zdiv;
    return zi < zalt ? p + (long long)zi * sz : alt + (long long)(zi - zalt) * sz;
  }
};

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kRKC = 32;   // k per chunk
constexpr int kRG = 2;     // chunks per register group

template <bool BF16> struct RLds {
  using T = typename std::conditional<BF16, __bf16, float>::type;
  static constexpr int LDT = BF16 ? 40 : 36;              // row stride of a transposition tile (elements)
  static constexpr int TILE = 32 * LDT;                   // one operand's 32 x 32 chunk
  static constexpr int WAVE = 2 * kRG * TILE;             // two operands for each chunk of a group
};

template <bool BF16> struct RFrag;
template <> struct RFrag<true> { bf16x8 v[2]; };
template <> struct RFrag<false> { float v[2][8]; };

// raw chunk of one operand: V = 1: raw[4 j + e] = row r0 + 8 j + lane / 8, k = k0 + 4 (lane % 8) + e;
// V = 0: raw[8 i + e] = row r0 + 16 i + li, k = k0 + 8 lq + e.  Rows past the end are
// clamped into the matrix (computed on valid data, never stored).  FULL: the chunk
// lies inside the contraction, else k >= kend reads as zero.
// One operand of one batch: rows at base (k < kalt) or kbase (k >= kalt, read at k - kalt).
struct ROp {
  const float* base; const float* kbase; long long lr, lk; int kalt;
};

template <int V, bool FULL>
__device__ __forceinline__ void rload(const ROp& m, float (&raw)[16], int r0, int rows, int k0, int kend, int lane) {
  const float* base = m.base;
  if (k0 >= m.kalt) {   // uniform: kalt is a multiple of the chunk
    base = m.kbase;
    k0 -= m.kalt;
    kend -= m.kalt;
  }
  if constexpr (V) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = min(r0 + 8 * j + (lane >> 3), rows - 1);
      const int kq = k0 + 4 * (lane & 7);
      const float* q = base + (long long)r * m.lr;
      if constexpr (FULL) {
        const f4v t = *reinterpret_cast<const f4v*>(__builtin_assume_aligned(q + kq, 16));
#pragma unroll
        for (int e = 0; e < 4; ++e) raw[4 * j + e] = t[e];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = kq + e;
          const float v = q[min(k, kend - 1)];   // kend > k0: always a valid element
          raw[4 * j + e] = k < kend ? v : 0.f;
        }
      }
    }
  } else {
    const int li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = min(r0 + 16 * i + li, rows - 1);
      const float* q = base + r * m.lr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * lq + e;
        if constexpr (FULL) {
          raw[8 * i + e] = q[(long long)k * m.lk];
        } else {
          const float v = q[(long long)min(k, kend - 1) * m.lk];
          raw[8 * i + e] = k < kend ? v : 0.f;
        }
      }
    }
  }
}

// raw chunk -> MFMA fragments.  V = 1 goes through the wave's LDS tile in two
// steps, so that the LDS round trips of a whole register group overlap: stage()
// writes the chunk, frag() reads the fragments back after the group's single wait.
template <bool BF16, int V>
__device__ __forceinline__ void stage(const float (&raw)[16], typename RLds<BF16>::T* tile, int lane) {
  using LL = RLds<BF16>;
  if constexpr (V) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      auto* dst = tile + (8 * j + (lane >> 3)) * LL::LDT + 4 * (lane & 7);
      if constexpr (BF16) {
        bf16x4 h;
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = (__bf16)raw[4 * j + e];
        *reinterpret_cast<bf16x4*>(dst) = h;
      } else {
        *reinterpret_cast<f4v*>(dst) = f4v{raw[4 * j], raw[4 * j + 1], raw[4 * j + 2], raw[4 * j + 3]};
      }
    }
  }
}

template <bool BF16, int V>
__device__ __forceinline__ void frag(const float (&raw)[16], const typename RLds<BF16>::T* tile, int lane,
                                     RFrag<BF16>& f) {
  using LL = RLds<BF16>;
  const int li = lane & 15, lq = lane >> 4;
  if constexpr (V) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const auto* src = tile + (16 * i + li) * LL::LDT + 8 * lq;
      if constexpr (BF16) {
        f.v[i] = *reinterpret_cast<const bf16x8*>(src);
      } else {
        const f4v a = *reinterpret_cast<const f4v*>(src), b = *reinterpret_cast<const f4v*>(src + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          f.v[i][e] = a[e];
          f.v[i][4 + e] = b[e];
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (BF16) f.v[i][e] = (__bf16)raw[8 * i + e];
        else f.v[i][e] = raw[8 * i + e];
      }
  }
}

// the wave's own LDS writes complete before any lane reads them back (and the
// compiler keeps every LDS access on its side of this point)
__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <bool BF16>
__device__ __forceinline__ void rmma(const RFrag<BF16>& a, const RFrag<BF16>& b, v4f (&acc)[2][2]) {
  if constexpr (BF16) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v[i], b.v[jj], acc[i][jj], 0, 0, 0);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[i][e], b.v[jj][e], acc[i][jj], 0, 0, 0);
  }
}

// The end of a tile: the four waves' partial tiles summed through LDS in a fixed
// order (the buffer overlays the waves' operand tiles), then the stores or the
// tile epilogue.  All threads call.
template <class ST, bool SPLIT>
__device__ __forceinline__ void tile_out(const v4f (&acc)[2][2], const ST& st, const StPart& sp, int M, int N, int m0,
                                         int n0, int z, int split, int wave, int lane, char* lds) {
  constexpr int RLD = kTile + 1;
  const int li = lane & 15, lq = lane >> 4;
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        red[(wave * kTile + i * 16 + 4 * lq + q) * RLD + j * 16 + li] = acc[i][j][q];
  __syncthreads();
  for (int e = threadIdx.x; e < kTile * kTile; e += kThreads) {
    const int r = e / kTile, c = e - r * kTile;
    const float v = ((red[(0 * kTile + r) * RLD + c] + red[(1 * kTile + r) * RLD + c]) +
                     red[(2 * kTile + r) * RLD + c]) + red[(3 * kTile + r) * RLD + c];
    const int gr = m0 + r, gc = n0 + c;
    if constexpr (ST::ROWS && !SPLIT) {
      red[r * RLD + c] = v;   // wave 0's slot of this element: read above by this thread only
    } else if (gr < M && gc < N) {
      if constexpr (SPLIT) sp.put(z, split, gr, gc, v); else st.put(z, gr, gc, v);
    }
  }
  if constexpr (ST::ROWS && !SPLIT) {
    __syncthreads();
    st.rows(m0, min(kTile, M - m0), red, RLD, red + kTile * RLD);
  }
}

template <bool BF16, int AV, int BV>
constexpr int gemm_lds_bytes() {
  using LL = RLds<BF16>;
  constexpr int RED_BYTES = 4 * kTile * (kTile + 1) * 4;
  constexpr int TILE_BYTES = (AV || BV) ? 4 * LL::WAVE * (int)sizeof(typename LL::T) : 0;
  return TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES;
}

// one 32 x 32 output tile (bx, by) of batch / split index bz
template <bool BF16, int AV, int BV, class ST, bool SPLIT>
__device__ __forceinline__ void gemm_tile(const RMat& fa, const RMat& fb, const ST& st, const StPart& sp, int M,
                                          int N, int K, int kchunk, int bx, int by, int bz, char* lds) {
  using LL = RLds<BF16>;
  using T = typename LL::T;
  constexpr int KC = kRKC, G = kRG;

  const int z = bz / (SPLIT ? sp.splits : 1);
  const int split = SPLIT ? bz % sp.splits : 0;
  const int m0 = bx * kTile, n0 = by * kTile;
  const ROp oa{fa.batch(z), fa.kp ? fa.kp + (long long)z * fa.sz : nullptr, fa.lr, fa.lk, fa.kalt};
  const ROp ob{fb.batch(z), fb.kp ? fb.kp + (long long)z * fb.sz : nullptr, fb.lr, fb.lk, fb.kalt};
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: chunk tests stay scalar
  T* wt = reinterpret_cast<T*>(lds) + wave * LL::WAVE;   // this wave's tiles: [chunk of the group][operand]
  // this wave's k range: a quarter of the workgroup's, in whole chunks
  const int span = kend > kbeg ? kend - kbeg : 0;
  const int per = ((span + 3) / 4 + KC - 1) / KC * KC;
  const int wb = kbeg + wave * per;
  const int we = min(kend, wb + per);
  const int wspan = we > wb ? we - wb : 0;
  const int ngf = wspan / KC / G;      // groups of G chunks wholly inside the range

  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  float ra[2][G][16], rb[2][G][16];
  auto load = [&](int g, int buf) {
#pragma unroll
    for (int c = 0; c < G; ++c) {
      rload<AV, true>(oa, ra[buf][c], m0, M, wb + (g * G + c) * KC, we, lane);
      rload<BV, true>(ob, rb[buf][c], n0, N, wb + (g * G + c) * KC, we, lane);
    }
  };
  // a group's chunks: stage all (V = 1), one wait, then fragments and products
  auto mult = [&](int buf) {
    if constexpr (AV || BV) {
#pragma unroll
      for (int c = 0; c < G; ++c) {
        stage<BF16, AV>(ra[buf][c], wt + (2 * c) * LL::TILE, lane);
        stage<BF16, BV>(rb[buf][c], wt + (2 * c + 1) * LL::TILE, lane);
      }
      lds_wave_sync();
    }
#pragma unroll
    for (int c = 0; c < G; ++c) {
      RFrag<BF16> fa_, fb_;
      frag<BF16, AV>(ra[buf][c], wt + (2 * c) * LL::TILE, lane, fa_);
      frag<BF16, BV>(rb[buf][c], wt + (2 * c + 1) * LL::TILE, lane, fb_);
      rmma<BF16>(fa_, fb_, acc);
    }
    if constexpr (AV || BV) asm volatile("" ::: "memory");
  };
  auto chunk = [&](const float (&a)[16], const float (&b)[16]) {
    RFrag<BF16> fa_, fb_;
    if constexpr (AV || BV) {
      stage<BF16, AV>(a, wt, lane);
      stage<BF16, BV>(b, wt + LL::TILE, lane);
      lds_wave_sync();
    }
    frag<BF16, AV>(a, wt, lane, fa_);
    frag<BF16, BV>(b, wt + LL::TILE, lane, fb_);
    rmma<BF16>(fa_, fb_, acc);
    if constexpr (AV || BV) asm volatile("" ::: "memory");
  };
  // two register groups in flight: group g + 1 loads while group g multiplies
  if (ngf > 0) load(0, 0);
  if (ngf > 1) load(1, 1);
  for (int g = 0; g < ngf; g += 2) {
    mult(0);
    if (g + 2 < ngf) load(g + 2, 0);
    if (g + 1 < ngf) {
      mult(1);
      if (g + 3 < ngf) load(g + 3, 1);
    }
  }
  // the rest of the range chunk by chunk, then the partial last chunk
  int k0 = wb + ngf * G * KC;
  for (; k0 + KC <= we; k0 += KC) {
    float ta[16], tb[16];
    rload<AV, true>(oa, ta, m0, M, k0, we, lane);
    rload<BV, true>(ob, tb, n0, N, k0, we, lane);
    chunk(ta, tb);
  }
  if (k0 < we) {
    float ta[16], tb[16];
    rload<AV, false>(oa, ta, m0, M, k0, we, lane);
    rload<BV, false>(ob, tb, n0, N, k0, we, lane);
    chunk(ta, tb);
  }

  tile_out<ST, SPLIT>(acc, st, sp, M, N, m0, n0, z, split, wave, lane, lds);
}

template <bool BF16, int AV, int BV, class ST, bool SPLIT>
__global__ __launch_bounds__(kThreads) void k_gemm_r(RMat fa, RMat fb, ST st, StPart sp, int M, int N, int K,
                                                     int kchunk) {
  __shared__ __attribute__((aligned(16))) char lds[gemm_lds_bytes<BF16, AV, BV>()];
  int bx, by, bz;
  tile_of(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), gridDim.x, gridDim.y, gridDim.z, bx, by,
          bz);
  gemm_tile<BF16, AV, BV, ST, SPLIT>(fa, fb, st, sp, M, N, K, kchunk, bx, by, bz, lds);
}

// Two independent products in one launch (the input and weight gradients of one
// layer): workgroups [0, tiles0) take problem 0 (A row-coalesced when AV0, else
// k-strided; k-strided B), the rest problem 1 (both k-strided).
struct RProb {
  RMat a, b; StMat st; int M, N, K, gx, gy;
};

template <bool BF16, int AV0>
__global__ __launch_bounds__(kThreads) void k_gemm_pair(RProb p0, RProb p1, int tiles0) {
  constexpr int L0 = gemm_lds_bytes<BF16, AV0, 0>(), L1 = gemm_lds_bytes<BF16, 0, 0>();
  __shared__ __attribute__((aligned(16))) char lds[L0 > L1 ? L0 : L1];
  const StPart none{nullptr, 0, 0, 1};
  int b = blockIdx.x;
  if (b < tiles0) {
    gemm_tile<BF16, AV0, 0, StMat, false>(p0.a, p0.b, p0.st, none, p0.M, p0.N, p0.K, p0.K, b % p0.gx,
                                          (b / p0.gx) % p0.gy, b / (p0.gx * p0.gy), lds);
  } else {
    b -= tiles0;
    gemm_tile<BF16, 0, 0, StMat, false>(p1.a, p1.b, p1.st, none, p1.M, p1.N, p1.K, p1.K, b % p1.gx,
                                        (b / p1.gx) % p1.gy, b / (p1.gx * p1.gy), lds);
  }
}

// Two independent forward products (both operands row-coalesced) in one launch,
// e.g. the actor's and the critics' input projections of the same features.
template <bool BF16>
__global__ __launch_bounds__(kThreads) void k_gemm_pair_f(RProb p0, RProb p1, int tiles0) {
  __shared__ __attribute__((aligned(16))) char lds[gemm_lds_bytes<BF16, 1, 1>()];
  const StPart none{nullptr, 0, 0, 1};
  int b = blockIdx.x;
  if (b < tiles0) {
    gemm_tile<BF16, 1, 1, StMat, false>(p0.a, p0.b, p0.st, none, p0.M, p0.N, p0.K, p0.K, b % p0.gx,
                                        (b / p0.gx) % p0.gy, b / (p0.gx * p0.gy), lds);
  } else {
    b -= tiles0;
    gemm_tile<BF16, 1, 1, StMat, false>(p1.a, p1.b, p1.st, none, p1.M, p1.N, p1.K, p1.K, b % p1.gx,
                                        (b / p1.gx) % p1.gy, b / (p1.gx * p1.gy), lds);
  }
}

// ---------------------------------------------------------------- bfloat16-stored operands
// Products whose two operands both have bfloat16 copies (written by the operands'
// producers) read the copies: 8 elements per 16-byte lane load, half the bytes and
// half the load instructions of the FP32 form, and no conversion.  The tile, the
// wave split of K, the chunk order, each lane's k positions in the fragments and
// the final sum are those of gemm_tile, so the result is the same bit for bit.
//
// An operand is read in one of two orientations:
//  - plain (k-contiguous rows): four lanes cover a row's 64 bytes of a chunk;
//  - transposed (rows contiguous, k strided -- dY and X of a weight gradient, W
//    of an input gradient): four lanes cover 32 rows at one k, and the chunk is
//    written transposed into the wave's LDS tile.
// Fragments are then read from the LDS tile; a transposed operand's tile swizzles
// its 16-byte k groups by row (group g of row c sits at g ^ (c / 8) mod 4), so the
// transposing stores of the 64 lanes spread over the banks.  DIRECT (both operands plain, short K
// ranges): lane (li, lq) loads its fragment (rows li and 16 + li, k = 8 lq ..
// 8 lq + 7 of the chunk) straight from memory.
typedef unsigned u4v __attribute__((ext_vector_type(4)));

struct HMat {
  const uint16_t* p; long long ld, sz;   // ld: between rows (plain) or between k (transposed)
  const uint16_t* alt; int zalt, zdiv;
  const uint16_t* kp; int kalt;          // k >= kalt read from kp (+ z sz) at k - kalt
  int lim;   // the last 8-element group start inside every line: k (plain) or row (transposed)
  __device__ __forceinline__ const uint16_t* batch(int z) const {
    const int zi = z / zdiv;
    return zi < zalt ? p + (long long)zi * sz : alt + (long long)(zi - zalt) * sz;
  }
};

constexpr int kHMaxC = 4;   // chunks of a wave in flight at once
constexpr int kHLdt = 40;   // row stride of a wave's LDS tile (elements)
constexpr int kHTile = 32 * kHLdt;

// element (c, k) of a wave's tile; a transposed operand's tile swizzles its 16-byte k groups
template <bool T>
__device__ __forceinline__ int hpos(int c, int k) {
  if constexpr (T) return c * kHLdt + ((((k >> 3) ^ (c >> 3)) & 3) << 3) + (k & 7);
  return c * kHLdt + k;
}

// elements k >= kend of a loaded group starting at kq read as zero
__device__ __forceinline__ u4v hmask(u4v v, int kq, int kend) {
  const int nv = kend - kq;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const unsigned keep = nv >= 2 * d + 2 ? 0xffffffffu : (nv == 2 * d + 1 ? 0x0000ffffu : 0u);
    v[d] &= keep;
  }
  return v;
}

// one operand's part of chunk k0: two 16-byte groups per lane, at clamped addresses
// (rows, k-slices and groups past the end reread valid data; hmask_chunk zeroes
// what lies past the K range)
template <bool DIRECT, bool T, bool KP>
__device__ __forceinline__ void hload(const HMat& m, const uint16_t* base, const uint16_t* kbase, int r0, int rows,
                                      int k0, int kend, int lane, u4v (&v)[2]) {
  if (KP && k0 >= m.kalt) {   // uniform: kalt is a multiple of the chunk
    base = kbase;
    k0 -= m.kalt;
    kend -= m.kalt;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if constexpr (T) {
      const int k = min(k0 + 16 * j + (lane >> 2), kend - 1);
      v[j] = *reinterpret_cast<const u4v*>(base + (long long)k * m.ld + min(r0 + 8 * (lane & 3), m.lim));
    } else {
      const int r = min(r0 + (DIRECT ? 16 * j + (lane & 15) : 16 * j + (lane >> 2)), rows - 1);
      const int kq = k0 + (DIRECT ? 8 * (lane >> 4) : 8 * (lane & 3));
      v[j] = *reinterpret_cast<const u4v*>(base + (long long)r * m.ld + min(kq, m.lim));
    }
  }
}

// the K range's partial last chunk: elements k >= kend read as zero
template <bool DIRECT, bool T>
__device__ __forceinline__ void hmask_chunk(u4v (&v)[2], int k0, int kend, int lane) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if constexpr (T) {
      if (k0 + 16 * j + (lane >> 2) >= kend) v[j] = u4v{0u, 0u, 0u, 0u};
    } else {
      v[j] = hmask(v[j], k0 + (DIRECT ? 8 * (lane >> 4) : 8 * (lane & 3)), kend);
    }
  }
}

// a loaded chunk into the wave's LDS tile, as [row][k]
template <bool T>
__device__ __forceinline__ void hstage(const u4v (&v)[2], uint16_t* tile, int lane) {
  const int q = lane & 3;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int r = 16 * j + (lane >> 2);   // plain: the row; transposed: the k
    if constexpr (T) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const unsigned w = v[j][e >> 1];
        tile[hpos<true>(8 * q + e, r)] = (uint16_t)((e & 1) ? (w >> 16) : (w & 0xffffu));
      }
    } else {
      *reinterpret_cast<u4v*>(tile + hpos<false>(r, 8 * q)) = v[j];
    }
  }
}

template <bool DIRECT>
constexpr int hgemm_lds_bytes() {
  constexpr int RED_BYTES = 4 * kTile * (kTile + 1) * 4;
  constexpr int TILE_BYTES = DIRECT ? 0 : 4 * 2 * 2 * kHTile * 2;
  return TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES;
}

template <bool DIRECT, bool TA, bool TB, bool KP, class ST>
__device__ __forceinline__ void gemm_tile_h(const HMat& fa, const HMat& fb, const ST& st, int M, int N, int K, int bx,
                                            int by, int bz, char* lds) {
  static_assert(!DIRECT || (!TA && !TB), "the direct form reads plain operands");
  constexpr int KC = kRKC;
  const int m0 = bx * kTile, n0 = by * kTile;
  const uint16_t* ab = fa.batch(bz);
  const uint16_t* bb = fb.batch(bz);
  const uint16_t* akp = KP ? fa.kp + (long long)bz * fa.sz : nullptr;
  const uint16_t* bkp = KP ? fb.kp + (long long)bz * fb.sz : nullptr;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lq = lane >> 4;
  // this wave's k range, as in gemm_tile: a quarter of K in whole chunks
  const int per = ((K + 3) / 4 + KC - 1) / KC * KC;
  const int wb = wave * per;
  const int we = min(K, wb + per);
  const int nch = we > wb ? (we - wb + KC - 1) / KC : 0;
  uint16_t* wt = reinterpret_cast<uint16_t*>(lds) + wave * (2 * 2 * kHTile);

  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int g = 0; g < nch; g += kHMaxC) {
    u4v ra[kHMaxC][2], rb[kHMaxC][2];
#pragma unroll
    for (int c = 0; c < kHMaxC; ++c) {
      if (g + c < nch) {
        const int k0 = wb + (g + c) * KC;
        hload<DIRECT, TA, KP>(fa, ab, akp, m0, M, k0, we, lane, ra[c]);
        hload<DIRECT, TB, KP>(fb, bb, bkp, n0, N, k0, we, lane, rb[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < kHMaxC; ++c) {
      const int k0 = wb + (g + c) * KC;
      if (g + c < nch && k0 + KC > we) {
        hmask_chunk<DIRECT, TA>(ra[c], k0, we, lane);
        hmask_chunk<DIRECT, TB>(rb[c], k0, we, lane);
      }
    }
    if constexpr (DIRECT) {
#pragma unroll
      for (int c = 0; c < kHMaxC; ++c) {
        if (g + c < nch) {
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
              acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ra[c][i]),
                                                                   __builtin_bit_cast(bf16x8, rb[c][jj]), acc[i][jj],
                                                                   0, 0, 0);
        }
      }
    } else {
      // two chunks per LDS round (the wave's tiles hold two chunks of both operands)
#pragma unroll
      for (int h = 0; h < kHMaxC; h += 2) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
          if (g + h + c2 < nch) {
            hstage<TA>(ra[h + c2], wt + (2 * c2) * kHTile, lane);
            hstage<TB>(rb[h + c2], wt + (2 * c2 + 1) * kHTile, lane);
          }
        }
        lds_wave_sync();
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
          if (g + h + c2 < nch) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              a[i] = *reinterpret_cast<const bf16x8*>(wt + (2 * c2) * kHTile + hpos<TA>(16 * i + li, 8 * lq));
              b[i] = *reinterpret_cast<const bf16x8*>(wt + (2 * c2 + 1) * kHTile + hpos<TB>(16 * i + li, 8 * lq));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int jj = 0; jj < 2; ++jj)
                acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[jj], acc[i][jj], 0, 0, 0);
          }
        }
        asm volatile("" ::: "memory");
      }
    }
  }
  const StPart none{nullptr, 0, 0, 1};
  tile_out<ST, false>(acc, st, none, M, N, m0, n0, bz, 0, wave, lane, lds);
}

// the form of a bfloat16-copy product: transposed B (1), transposed A (2), the
// direct form (4), k-concatenated operands (8)
template <int FORM> struct HForm {
  static constexpr bool D = (FORM & 4) != 0, TA = (FORM & 2) != 0, TB = (FORM & 1) != 0, KP = (FORM & 8) != 0;
};
constexpr int kHDirect = 4, kHKp = 8;

template <int FORM, class ST>
__global__ __launch_bounds__(kThreads) void k_gemm_h(HMat fa, HMat fb, ST st, int M, int N, int K) {
  using F = HForm<FORM>;
  __shared__ __attribute__((aligned(16))) char lds[hgemm_lds_bytes<F::D>()];
  int bx, by, bz;
  tile_of(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), gridDim.x, gridDim.y, gridDim.z, bx, by,
          bz);
  gemm_tile_h<F::D, F::TA, F::TB, F::KP, ST>(fa, fb, st, M, N, K, bx, by, bz, lds);
}

// two products on bfloat16 copies in one launch (the forward pair of k_gemm_pair_f,
// or a layer's input and weight gradients as in k_gemm_pair)
struct HProb {
  HMat a, b; StMat st; int M, N, K, gx, gy;
};

template <int F0, int F1>
__global__ __launch_bounds__(kThreads) void k_gemm_pair_h(HProb p0, HProb p1, int tiles0) {
  using G0 = HForm<F0>;
  using G1 = HForm<F1>;
  constexpr int L0 = hgemm_lds_bytes<G0::D>(), L1 = hgemm_lds_bytes<G1::D>();
  __shared__ __attribute__((aligned(16))) char lds[L0 > L1 ? L0 : L1];
  int b = blockIdx.x;
  if (b < tiles0) {
    gemm_tile_h<G0::D, G0::TA, G0::TB, G0::KP, StMat>(p0.a, p0.b, p0.st, p0.M, p0.N, p0.K, b % p0.gx,
                                                      (b / p0.gx) % p0.gy, b / (p0.gx * p0.gy), lds);
  } else {
    b -= tiles0;
    gemm_tile_h<G1::D, G1::TA, G1::TB, G1::KP, StMat>(p1.a, p1.b, p1.st, p1.M, p1.N, p1.K, b % p1.gx,
                                                      (b / p1.gx) % p1.gy, b / (p1.gx * p1.gy), lds);
  }
}

// rows of a small matrix copied into another's columns, and into its bfloat16 copy
// when it has one (the unfused policy head's second action copy)
__global__ void k_copy_rows(const float* __restrict__ src, int cols, int rows, float* __restrict__ dst, long long ld,
                            uint16_t* __restrict__ dst_h) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int r = e / cols, c = e - r * cols;
  const float v = src[e];
  dst[(long long)r * ld + c] = v;
  if (dst_h) dst_h[(long long)r * ld + c] = bf16_bits(v);
}

// sum of split-K partials in split order, then the real store
template <class ST>
__global__ void k_split_reduce(StPart sp, ST st, int batch) {
  const long long MN = (long long)sp.M * sp.N;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= MN * batch) return;
  const int z = (int)(e / MN);
  const long long rc = e - z * MN;
  const int r = (int)(rc / sp.N), c = (int)(rc - (long long)r * sp.N);
  const float* p = sp.part + (long long)z * sp.splits * MN + rc;
  float v = 0.f;
  for (int s = 0; s < sp.splits; ++s) v += p[s * MN];
  st.put(z, r, c, v);
}

template <class FA, class FB, class ST>
static int run(int bf16, int M, int N, int K, int batch, FA fa, FB fb, ST st, float* scratch,
               size_t scratch_floats, hipStream_t stream, const char* what) {
  if (M <= 0 || N <= 0 || batch <= 0) return SQ_OK;
  const int bk = bf16 ? 4 * Cfg<true>::KW : 4 * Cfg<false>::KW;
  const int tiles = cdiv(M, kTile) * cdiv(N, kTile) * batch;
  int splits = 1;
  if (scratch && tiles < 192 && K > 8 * bk) {
    splits = cdiv(256, tiles);
    const int most = K / (2 * bk);
    splits = splits < most ? splits : most;
    while (splits > 1 && (size_t)splits * M * N * batch > scratch_floats) --splits;
  }
  int kchunk = K > 0 ? K : 1;
  if (splits > 1) {
    kchunk = cdiv(cdiv(K, splits), bk) * bk;
    splits = cdiv(K, kchunk);
  }
  StPart sp{scratch, M, N, splits};
  dim3 grid(cdiv(M, kTile), cdiv(N, kTile), batch * splits);
  if (splits <= 1) {
    if (bf16)
      k_gemm<true, FA, FB, ST, false><<<grid, kThreads, 0, stream>>>(fa, fb, st, sp, M, N, K, kchunk);
    else
      k_gemm<false, FA, FB, ST, false><<<grid, kThreads, 0, stream>>>(fa, fb, st, sp, M, N, K, kchunk);
    return launch_status(what);
  }
  if (bf16)
    k_gemm<true, FA, FB, ST, true><<<grid, kThreads, 0, stream>>>(fa, fb, st, sp, M, N, K, kchunk);
  else
    k_gemm<false, FA, FB, ST, true><<<grid, kThreads, 0, stream>>>(fa, fb, st, sp, M, N, K, kchunk);
  SQ_TRY(launch_status(what));
  const long long total = (long long)M * N * batch;
  k_split_reduce<ST><<<cdiv(total, 256), 256, 0, stream>>>(sp, st, batch);
  return launch_status("split_reduce");
}

// ---------------------------------------------------------------- public launchers
// 1: k is the contiguous dimension of 16-byte aligned rows (vector loads), else 0
static int rkind(const MatArg& a) {
  return ((uintptr_t)a.p % 16 == 0 && (!a.alt || (uintptr_t)a.alt % 16 == 0) &&
          (!a.kp || (uintptr_t)a.kp % 16 == 0) && a.sz % 4 == 0 && a.lk == 1 && a.lr % 4 == 0) ? 1 : 0;
}

static RMat rmat(const MatArg& m) { return RMat{m.p, m.lr, m.lk, m.sz, m.alt, m.zalt, m.zdiv, m.kp, m.kalt}; }
static StMat stmat(const OutArg& c) {
  return StMat{c.p, c.ld, c.sz, c.bias, c.bias_sz, c.accumulate, c.relu, c.bias_alt, c.bias_zalt};
}

// A product on the FP32 values of an operand whose owner keeps only its bfloat16
// copy would read stale data: refuse it (the copy-reading form did not apply).
static bool fp32_ok(const MatArg& m) {
  return !fp32_dropped(m.p) && !(m.alt && fp32_dropped(m.alt)) && !(m.kp && fp32_dropped(m.kp));
}
static int refuse_dropped(const char* what) {
  set_error("%s: an operand keeps only its bfloat16 copy, which this product's shape cannot read", what);
  return SQ_EINVAL;
}

// the K split gemm() would choose (1: none)
static int want_splits(int M, int N, int K, int batch, const float* scratch, size_t scratch_floats) {
  const int tiles = cdiv(M, kTile) * cdiv(N, kTile) * batch;
  int splits = 1;
  if (scratch && tiles < 128 && K >= 2048) {
    splits = std::min(cdiv(256, tiles), K / 1024);
    while (splits > 1 && (size_t)splits * M * N * batch > scratch_floats) --splits;
  }
  return splits;
}

// The bfloat16 copy of operand m of a product (`rows` rows, contraction K, `batch`
// batches) when every batch it reads has one, in one of the two orientations:
// plain (k-contiguous rows) or transposed (rows contiguous, k strided; *t set).
// Lines (rows, or k-slices) must be 16-byte aligned and hold the rounded-up
// extent the loads touch; a k-concatenated operand (kp) needs whole chunks on
// both sides of kalt.
static bool hmat(const MatArg& m, int rows, int K, int batch, HMat* out, bool* t) {
  const bool plain = m.lk == 1, trans = m.lr == 1 && m.lk > 1;
  if ((!plain && !trans) || rows <= 0 || K <= 0 || batch <= 0 || m.sz % 8) return false;
  const long long ld = plain ? m.lr : m.lk;
  if (ld % 8) return false;
  const bool kp = m.kp != nullptr;
  if (kp && (m.kalt <= 0 || m.kalt >= K || m.kalt % kRKC || (K - m.kalt) % kRKC)) return false;
  const long long kfirst = kp ? m.kalt : K, ksecond = kp ? K - m.kalt : 0;
  auto r8 = [](long long x) { return (x + 7) / 8 * 8; };
  long long len, ext_p, ext_kp;
  if (plain) {
    len = r8(std::max(kfirst, ksecond));
    ext_p = (long long)(rows - 1) * ld + len;
    ext_kp = ext_p;
  } else {
    len = r8(rows);
    ext_p = (kfirst - 1) * ld + len;
    ext_kp = (ksecond - 1) * ld + len;
  }
  if (ld < len) return false;
  const int nb = cdiv(batch, m.zdiv);
  const int np = std::min(nb, m.zalt);
  auto ok = [](const uint16_t* h) { return h && (uintptr_t)h % 16 == 0; };
  const uint16_t* hp = np > 0 ? twin_of(m.p, (long long)(np - 1) * m.sz + ext_p) : nullptr;
  if (np > 0 && !ok(hp)) return false;
  const uint16_t* ha = nullptr;
  if (nb > np) {
    ha = twin_of(m.alt, (long long)(nb - np - 1) * m.sz + ext_p);
    if (!ok(ha)) return false;
  }
  const uint16_t* hk = nullptr;
  if (kp) {
    hk = twin_of(m.kp, (long long)(batch - 1) * m.sz + ext_kp);
    if (!ok(hk)) return false;
  }
  *out = HMat{hp, ld, m.sz, ha, m.zalt, m.zdiv, hk, kp ? m.kalt : kNoAlt, (int)(len - 8)};
  *t = trans;
  return true;
}

// the direct load form for plain operands and short per-wave K ranges (at most three
// chunks); kp: an operand is k-concatenated
static int hform(bool ta, bool tb, int K, bool kp = false) {
  if (!ta && !tb && !kp && cdiv(cdiv(K, 4), kRKC) <= 3) return kHDirect;
  return (ta ? 2 : 0) | (tb ? 1 : 0) | (kp ? kHKp : 0);
}
static bool hkp(const HMat& a, const HMat& b) { return a.kp != nullptr || b.kp != nullptr; }

template <int FORM, class ST>
static void launch_h(dim3 grid, const HMat& a, const HMat& b, const ST& out, int M, int N, int K, hipStream_t st) {
  k_gemm_h<FORM, ST><<<grid, kThreads, 0, st>>>(a, b, out, M, N, K);
}

template <class ST>
static int run_h(int form, dim3 grid, const HMat& a, const HMat& b, const ST& out, int M, int N, int K,
                 hipStream_t st) {
  switch (form) {
    case 0: launch_h<0>(grid, a, b, out, M, N, K, st); break;
    case 1: launch_h<1>(grid, a, b, out, M, N, K, st); break;
    case 2: launch_h<2>(grid, a, b, out, M, N, K, st); break;
    case 3: launch_h<3>(grid, a, b, out, M, N, K, st); break;
    case kHDirect: launch_h<kHDirect>(grid, a, b, out, M, N, K, st); break;
    case kHKp | 1: launch_h<kHKp | 1>(grid, a, b, out, M, N, K, st); break;
    default: return kNotApplicable;
  }
  note_copy_product();
  return launch_status("gemm_h");
}

// the product on bfloat16 copies when both operands have them (kNotApplicable: not eligible)
static int try_h(int M, int N, int K, int batch, const MatArg& A, const MatArg& B, const StMat& out, hipStream_t st) {
  HMat ha, hb;
  bool ta, tb;
  if (!hmat(A, M, K, batch, &ha, &ta) || !hmat(B, N, K, batch, &hb, &tb)) return kNotApplicable;
  return run_h(hform(ta, tb, K, hkp(ha, hb)), dim3(cdiv(M, kTile), cdiv(N, kTile), batch), ha, hb, out, M, N, K, st);
}

// an operand given as bfloat16 bits: plain (lk == 1) or transposed (lr == 1)
static bool hraw(const uint16_t* p, long long lr, long long lk, long long sz, int rows, int K, HMat* out, bool* t) {
  const bool plain = lk == 1, trans = lr == 1 && lk > 1;
  const long long ld = plain ? lr : lk, len = plain ? (K + 7) / 8 * 8 : (rows + 7) / 8 * 8;
  if ((!plain && !trans) || !p || (uintptr_t)p % 16 || ld % 8 || sz % 8 || ld < len) return false;
  *out = HMat{p, ld, sz, nullptr, kNoAlt, 1, nullptr, kNoAlt, (int)(len - 8)};
  *t = trans;
  return true;
}

int gemm_bf16_stored(int M, int N, int K, int batch, const uint16_t* A, long long a_lr, long long a_lk,
                     long long a_sz, const uint16_t* B, long long b_lr, long long b_lk, long long b_sz, OutArg C,
                     hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return SQ_OK;
  HMat a, b;
  bool ta, tb;
  if (K <= 0 || !C.p || !hraw(A, a_lr, a_lk, a_sz, M, K, &a, &ta) || !hraw(B, b_lr, b_lk, b_sz, N, K, &b, &tb)) {
    set_error("gemm_bf16: each operand needs k-contiguous rows (or contiguous rows, k strided), 16-byte aligned, "
              "of at least K (or its rows) rounded up to 8 elements");
    return SQ_EINVAL;
  }
  return run_h(hform(ta, tb, K), dim3(cdiv(M, kTile), cdiv(N, kTile), batch), a, b, stmat(C), M, N,
               K, st);
}

template <bool BF16, int AV, int BV>
static int run_r(int M, int N, int K, int batch, const MatArg& A, const MatArg& B, const StMat& out, float* scratch,
                 size_t scratch_floats, hipStream_t st) {
  // few output tiles over a long contraction: split K across workgroups
  int splits = want_splits(M, N, K, batch, scratch, scratch_floats);
  int kchunk = K > 0 ? K : 1;
  if (splits > 1) {
    kchunk = cdiv(cdiv(K, splits), 4 * kRKC) * 4 * kRKC;
    splits = cdiv(K, kchunk);
  }
  const RMat a = rmat(A), b = rmat(B);
  StPart sp{scratch, M, N, splits};
  dim3 grid(cdiv(M, kTile), cdiv(N, kTile), batch * splits);
  if (splits <= 1) {
    k_gemm_r<BF16, AV, BV, StMat, false><<<grid, kThreads, 0, st>>>(a, b, out, sp, M, N, K, kchunk);
    return launch_status("gemm");
  }
  k_gemm_r<BF16, AV, BV, StMat, true><<<grid, kThreads, 0, st>>>(a, b, out, sp, M, N, K, kchunk);
  SQ_TRY(launch_status("gemm_split"));
  const long long total = (long long)M * N * batch;
  k_split_reduce<StMat><<<cdiv(total, 256), 256, 0, st>>>(sp, out, batch);
  return launch_status("split_reduce");
}

int gemm(int bf16, int M, int N, int K, int batch, MatArg A, MatArg B, OutArg C, float* scratch,
         size_t scratch_floats, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return SQ_OK;
  if ((A.kalt != kNoAlt && A.kalt % kRKC) || (B.kalt != kNoAlt && B.kalt % kRKC) || A.kalt != B.kalt) {
    set_error("gemm: a k-split operand needs the same kalt on both sides, a multiple of %d", kRKC);
    return SQ_EINVAL;
  }
  const StMat out = stmat(C);
  const int va = rkind(A), vb = rkind(B);
  // the copy form does not split K; an operand without FP32 values takes it unsplit
  const bool fp32 = fp32_ok(A) && fp32_ok(B);
  if (bf16 && (!fp32 || want_splits(M, N, K, batch, scratch, scratch_floats) == 1)) {
    const int h = try_h(M, N, K, batch, A, B, out, st);
    if (h != kNotApplicable) return h;
  }
  if (!fp32) return refuse_dropped("gemm");
  if (bf16) {
    if (va && vb) return run_r<true, 1, 1>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
    if (va) return run_r<true, 1, 0>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
    if (vb) return run_r<true, 0, 1>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
    return run_r<true, 0, 0>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
  }
  if (va && vb) return run_r<false, 1, 1>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
  if (va) return run_r<false, 1, 0>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
  if (vb) return run_r<false, 0, 1>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
  return run_r<false, 0, 0>(M, N, K, batch, A, B, out, scratch, scratch_floats, st);
}

int gemm_tanh_gauss(int bf16, int n, int A, int K, MatArg X, MatArg W, const float* bias, const float* eps, float lo,
                    float hi, float* action, float* logp, float* save, float* head, hipStream_t st, float* xact,
                    long long ld_xact, int xact_row0) {
  if (n <= 0) return SQ_OK;
  if (2 * A > kTile || rkind(X) != 1 || rkind(W) != 1 || !head) {
    OutArg C{head, 2 * A, 0, bias, 0, 0, 0};
    if (!head) {
      set_error("gemm_tanh_gauss: the unfused form needs the head buffer");
      return SQ_EINVAL;
    }
    SQ_TRY(gemm(bf16, n, 2 * A, K, 1, X, W, C, nullptr, 0, st));
    SQ_TRY(eps ? tanh_gauss_fwd(head, n, A, eps, lo, hi, action, logp, save, st)
               : mean_action(head, n, A, action, st));
    if (xact && xact_row0 < n) {
      const int rows = n - xact_row0;
      k_copy_rows<<<cdiv((long long)rows * A, 256), 256, 0, st>>>(action + (size_t)xact_row0 * A, A, rows, xact,
                                                                   ld_xact, twin_of(xact, (rows - 1) * ld_xact + A));
      return launch_status("copy_rows");
    }
    return SQ_OK;
  }
  uint16_t* xact_h = xact && xact_row0 < n ? twin_of(xact, (long long)(n - xact_row0 - 1) * ld_xact + A) : nullptr;
  const StTanhGauss tg{bias, eps, lo, hi, action, logp, save, head, A, xact, ld_xact, xact_row0, xact_h};
  const StPart none{nullptr, 0, 0, 1};
  dim3 grid(cdiv(n, kTile), 1, 1);
  HMat hx, hw;
  bool tx, tw;
  if (bf16 && hmat(X, n, K, 1, &hx, &tx) && hmat(W, 2 * A, K, 1, &hw, &tw) && !tx && !tw && !hkp(hx, hw)) {
    if (hform(false, false, K) == kHDirect) launch_h<kHDirect>(grid, hx, hw, tg, n, 2 * A, K, st);
    else launch_h<0>(grid, hx, hw, tg, n, 2 * A, K, st);
    note_copy_product();
    return launch_status("gemm_tanh_gauss");
  }
  if (!fp32_ok(X) || !fp32_ok(W)) return refuse_dropped("gemm_tanh_gauss");
  if (bf16)
    k_gemm_r<true, 1, 1, StTanhGauss, false><<<grid, kThreads, 0, st>>>(rmat(X), rmat(W), tg, none, n, 2 * A, K, K);
  else
    k_gemm_r<false, 1, 1, StTanhGauss, false><<<grid, kThreads, 0, st>>>(rmat(X), rmat(W), tg, none, n, 2 * A, K, K);
  return launch_status("gemm_tanh_gauss");
}

int gemm_tg_bwd(int bf16, const GemmProb& dx, int A, const TgBwdJob& tg, hipStream_t st) {
  const int n = dx.M;
  if (n <= 0) return SQ_OK;
  const int ldh = tg.ldh > 0 ? tg.ldh : 2 * A;
  const bool kok = dx.A.kalt == dx.B.kalt && (dx.A.kalt == kNoAlt || dx.A.kalt % kRKC == 0);
  if (dx.N != A || 2 * A * kTile > kTile * kTile || dx.batch != 1 || rkind(dx.A) != 1 || rkind(dx.B) != 0 || !kok ||
      dx.C.accumulate || dx.C.bias) {
    SQ_TRY(gemm(bf16, dx.M, dx.N, dx.K, dx.batch, dx.A, dx.B, dx.C, nullptr, 0, st));
    return tanh_gauss_bwd(tg.save, tg.eps, dx.C.p, dx.C.ld, tg.dlogp_vec, tg.dlogp_scalar, tg.scale, tg.lo, tg.hi, n,
                          A, tg.dhead, tg.part, st, ldh);
  }
  uint16_t* dhead_h = twin_of(tg.dhead, (long long)(n - 1) * ldh + 2 * A);
  StTgBwd ep{tg.save, tg.eps, tg.dlogp_vec, tg.dlogp_scalar, tg.scale, tg.lo, tg.hi, tg.dhead, tg.part, A,
             ldh, dhead_h, 0};
  const StPart none{nullptr, 0, 0, 1};
  dim3 grid(cdiv(n, kTile), 1, 1);
  HMat ha, hb;
  bool ta, tb;
  if (bf16 && hmat(dx.A, n, dx.K, 1, &ha, &ta) && !ta) {
    // on bfloat16 copies the product reads da's weight columns from the 16-byte
    // aligned group that holds them: the window starts `off` columns earlier and
    // the epilogue skips them
    for (int off = 0; off < 8 && A + off <= kTile; ++off) {
      MatArg bw = dx.B;
      bw.p -= off;
      if (bw.kp) bw.kp -= off;
      if (!hmat(bw, A + off, dx.K, 1, &hb, &tb) || !tb) continue;
      ep.off = off;
      if (hkp(ha, hb)) launch_h<kHKp | 1>(grid, ha, hb, ep, n, A + off, dx.K, st);
      else launch_h<1>(grid, ha, hb, ep, n, A + off, dx.K, st);
      note_copy_product();
      return launch_status("gemm_tg_bwd");
    }
  }
  if (!fp32_ok(dx.A) || !fp32_ok(dx.B)) return refuse_dropped("gemm_tg_bwd");
  if (bf16)
    k_gemm_r<true, 1, 0, StTgBwd, false><<<grid, kThreads, 0, st>>>(rmat(dx.A), rmat(dx.B), ep, none, n, A, dx.K,
                                                                     dx.K);
  else
    k_gemm_r<false, 1, 0, StTgBwd, false><<<grid, kThreads, 0, st>>>(rmat(dx.A), rmat(dx.B), ep, none, n, A, dx.K,
                                                                      dx.K);
  return launch_status("gemm_tg_bwd");
}

int gemm_pair(int bf16, const GemmProb& p0, const GemmProb& p1, float* scratch, size_t scratch_floats,
              hipStream_t st) {
  const bool e0 = p0.M <= 0 || p0.N <= 0 || p0.batch <= 0, e1 = p1.M <= 0 || p1.N <= 0 || p1.batch <= 0;
  // (input gradient, weight gradient) of a layer, or two forward products
  const bool grad_kinds = rkind(p0.B) == 0 && rkind(p1.A) == 0 && rkind(p1.B) == 0;
  const bool fwd_kinds = rkind(p0.A) == 1 && rkind(p0.B) == 1 && rkind(p1.A) == 1 && rkind(p1.B) == 1;
  const bool kinds = grad_kinds || fwd_kinds;
  const bool nosplit = want_splits(p0.M, p0.N, p0.K, p0.batch, scratch, scratch_floats) == 1 &&
                       want_splits(p1.M, p1.N, p1.K, p1.batch, scratch, scratch_floats) == 1;
  const bool kok = p0.A.kalt == p0.B.kalt && p1.A.kalt == p1.B.kalt &&
                   (p0.A.kalt == kNoAlt || p0.A.kalt % kRKC == 0) && (p1.A.kalt == kNoAlt || p1.A.kalt % kRKC == 0);
  if (e0 || e1 || !kinds || !nosplit || !kok) {
    SQ_TRY(gemm(bf16, p0.M, p0.N, p0.K, p0.batch, p0.A, p0.B, p0.C, scratch, scratch_floats, st));
    return gemm(bf16, p1.M, p1.N, p1.K, p1.batch, p1.A, p1.B, p1.C, scratch, scratch_floats, st);
  }
  RProb q0{rmat(p0.A), rmat(p0.B), stmat(p0.C), p0.M, p0.N, p0.K, cdiv(p0.M, kTile),
           cdiv(p0.N, kTile)};
  RProb q1{rmat(p1.A), rmat(p1.B), stmat(p1.C), p1.M, p1.N, p1.K, cdiv(p1.M, kTile),
           cdiv(p1.N, kTile)};
  const int t0 = q0.gx * q0.gy * p0.batch, t1 = q1.gx * q1.gy * p1.batch;
  HMat h0a, h0b, h1a, h1b;
  bool s0a, s0b, s1a, s1b;
  if (bf16 && hmat(p0.A, p0.M, p0.K, p0.batch, &h0a, &s0a) && hmat(p0.B, p0.N, p0.K, p0.batch, &h0b, &s0b) &&
      hmat(p1.A, p1.M, p1.K, p1.batch, &h1a, &s1a) && hmat(p1.B, p1.N, p1.K, p1.batch, &h1b, &s1b)) {
    const HProb r0{h0a, h0b, q0.st, p0.M, p0.N, p0.K, q0.gx, q0.gy};
    const HProb r1{h1a, h1b, q1.st, p1.M, p1.N, p1.K, q1.gx, q1.gy};
    const int f0 = hform(s0a, s0b, p0.K, hkp(h0a, h0b)), f1 = hform(s1a, s1b, p1.K, hkp(h1a, h1b));
    bool done = true;
    if (f0 == kHDirect && f1 == kHDirect) k_gemm_pair_h<kHDirect, kHDirect><<<t0 + t1, kThreads, 0, st>>>(r0, r1, t0);
    else if (f0 == 1 && f1 == 3) k_gemm_pair_h<1, 3><<<t0 + t1, kThreads, 0, st>>>(r0, r1, t0);
    else if (f0 == (kHKp | 1) && f1 == 3) k_gemm_pair_h<kHKp | 1, 3><<<t0 + t1, kThreads, 0, st>>>(r0, r1, t0);
    else if ((f0 == 0 || f0 == kHDirect) && (f1 == 0 || f1 == kHDirect))
      k_gemm_pair_h<0, 0><<<t0 + t1, kThreads, 0, st>>>(r0, r1, t0);
    else done = false;
    if (done) {
      note_copy_product();
      return launch_status("gemm_pair_h");
    }
  }
  if (!fp32_ok(p0.A) || !fp32_ok(p0.B) || !fp32_ok(p1.A) || !fp32_ok(p1.B)) return refuse_dropped("gemm_pair");
  if (fwd_kinds) {
    if (bf16) k_gemm_pair_f<true><<<t0 + t1, kThreads, 0, st>>>(q0, q1, t0);
    else k_gemm_pair_f<false><<<t0 + t1, kThreads, 0, st>>>(q0, q1, t0);
  } else {
    const int av0 = rkind(p0.A);
    if (bf16 && av0) k_gemm_pair<true, 1><<<t0 + t1, kThreads, 0, st>>>(q0, q1, t0);
    else if (bf16) k_gemm_pair<true, 0><<<t0 + t1, kThreads, 0, st>>>(q0, q1, t0);
    else if (av0) k_gemm_pair<false, 1><<<t0 + t1, kThreads, 0, st>>>(q0, q1, t0);
    else k_gemm_pair<false, 0><<<t0 + t1, kThreads, 0, st>>>(q0, q1, t0);
  }
  return launch_status("gemm_pair");
}

template <class F>
static int with_geo(int H, int Ho, int stride, F&& f) {
  if (H == 16 && Ho == 7 && stride == 2) return f(Geo<16, 7, 2>{16, 7, 2});
  if (H == 7 && Ho == 5 && stride == 1) return f(Geo<7, 5, 1>{7, 5, 1});
  if (H == 5 && Ho == 3 && stride == 1) return f(Geo<5, 3, 1>{5, 3, 1});
  return f(Geo<0, 0, 0>{H, Ho, stride});
}

int conv_fwd(int bf16, const float* x, int n, int Cin, int H, int stride, const float* W, const float* b, int F,
             float* out, hipStream_t st) {
  const int Ho = (H - 3) / stride + 1;
  const int K = Cin * 9;
  return with_geo(H, Ho, stride, [&](auto g) {
    using G = decltype(g);
    FConvPatch<G> fa{x, Cin, g};
    FMat<true> fb{W, K, 1, 0};
    StConv sc{out, F, Ho * Ho, b, 1};
    return run(bf16, n * Ho * Ho, F, K, 1, fa, fb, sc, nullptr, 0, st, "conv_fwd");
  });
}

size_t conv_dw_scratch_floats(int n, int Cin, int H, int stride, int F) {
  (void)n; (void)H; (void)stride;
  return (size_t)256 * F * (Cin * 9);
}

int conv_dw(int bf16, const float* x, int n, int Cin, int H, int stride, const float* dout, const float* out,
            int F, float* dW, float* part, size_t part_floats, hipStream_t st) {
  const int Ho = (H - 3) / stride + 1;
  const int K = Cin * 9;
  return with_geo(H, Ho, stride, [&](auto g) {
    using G = decltype(g);
    FConvGradT<G> fa{dout, out, F, g};
    FConvPatchT<G> fb{FConvPatch<G>{x, Cin, g}};
    StMat sm{dW, K, 0, nullptr, 0, 0, 0};
    return run(bf16, F, K, n * Ho * Ho, 1, fa, fb, sm, part, part_floats, st, "conv_dw");
  });
}

int conv_dx(int bf16, const float* dout, const float* out, int n, int Cin, int H, const float* W, int F, float* dx,
            hipStream_t st) {
  const int Ho = H - 2;
  return with_geo(H, Ho, 1, [&](auto g) {
    using G = decltype(g);
    FConvDxA<G> fa{dout, out, F, g};
    FConvDxB fb{W, Cin};
    StConv sc{dx, Cin, H * H, nullptr, 0};
    return run(bf16, n * H * H, Cin, F * 9, 1, fa, fb, sc, nullptr, 0, st, "conv_dx");
  });
}

}  // namespace sq
