// Adam with bias correction, fused with the target-critic EMA (Alg. 1 target
// update) and an optional bfloat16 copy of the new parameters.  One flat launch
// covers a whole optimiser group (encoder + critic, or actor).
#include <math.h>

#include "../common.h"
#include "bf16.h"
#include "finish.h"

namespace sq {

// the packed position of flat index i (relative to the optimiser's range), or -1
__device__ __forceinline__ long long pack_pos(const PackArgs& pk, long long i, int* critic) {
  const long long gi = i + pk.p_begin;
  for (int s = 0; s < pk.n; ++s) {
    const PackSeg& q = pk.seg[s];
    const long long loc = gi - q.src;
    if (loc >= 0 && loc < (long long)q.rows * q.cols) {
      const long long r = loc / q.cols;
      *critic = q.critic;
      return q.dst + r * q.ldp + (loc - r * q.cols);
    }
  }
  return -1;
}

// Each workgroup updates 256 * PER consecutive parameters (PER = 4, or 2 where
// that leaves fewer than kAdamMinPerCU element workgroups per compute unit: the
// actor's launch measured 10.2 against 11.4 us with 2, the critic's 20.3 against
// 18.1 us).  The packed segment holding the workgroup's first parameter is found
// once; parameters of that segment map to their packed position with one
// division, the rare others (a workgroup straddling a segment boundary) search
// the table.  Gradients given as row-block partials (gs) are summed here, in row
// order.  Every parameter's update is independent, so PER changes no result.
constexpr int kAdamCUs = 256, kAdamMinPerCU = 3;

// fixed-order sum over the 256 threads; valid in thread 0
__device__ float adam_block_sum(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// Temperature step (Sec. III learned temperature; Alg. 1): L = alpha * mean(-log pi
// - target entropy), so d L / d log alpha is the same value; one Adam step on log
// alpha with step ctr[CTR_TALPHA] + 1.  scal: [0] alpha before, [1] alpha after,
// [2] L_alpha, [3] mean entropy.
__device__ void alpha_block(const AlphaJob& j, float lr, float b1, float b2, float eps) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < j.B; i += 256) s += j.logp[i];
  s = adam_block_sum(s, sh);
  if (threadIdx.x != 0) return;
  const float ent = -s / (float)j.B;
  const float la = *j.log_alpha;
  const float alpha = expf(la);
  const float gr = alpha * (ent - j.target_entropy);
  const float t = (float)(j.ctr[CTR_TALPHA] + 1);
  const float mm = b1 * (*j.m) + (1.f - b1) * gr;
  const float vv = b2 * (*j.v) + (1.f - b2) * gr * gr;
  const float mh = mm / (1.f - powf(b1, t));
  const float vh = vv / (1.f - powf(b2, t));
  const float la2 = la - lr * mh / (sqrtf(vh) + eps);
  *j.m = mm;
  *j.v = vv;
  *j.log_alpha = la2;
  if (j.grad) *j.grad = gr;
  if (j.step_snap) *j.step_snap = j.ctr[CTR_TA];
  j.scal[0] = alpha;
  j.scal[1] = expf(la2);
  j.scal[2] = gr;
  j.scal[3] = ent;
}


struct AdamArgs {
  float* p; const float* g; float* m; float* v; long long n;
  float lr, b1, b2, eps;
  const int* step; float* ema; long long ema_begin; float rho; uint16_t* shadow;
  EncPrepMap ep;   // ep.n == 0: no prepared encoder copy to refresh
};

// conv weight i (updated to v) in the fused encoder's prepared copy
// (bfloat16 form: packed bfloat16 elements at the same element offsets)
__device__ __forceinline__ void enc_prep_put(const EncPrepMap& e, long long i, float v) {
  uint16_t* wb = reinterpret_cast<uint16_t*>(e.wp);
  const uint16_t vb = bf16_bits(v);
  for (int l = 0; l < e.n; ++l) {
    const long long o = i - e.W[l];
    if (o < 0 || o >= (long long)e.F * e.cin[l] * 9) continue;
    const int oi = (int)o, k = e.cin[l] * 9;
    const int f = oi / k, r = oi - f * k, c = r / 9, tap = r - 9 * c;
    const long long fo = e.fb[l] + (long long)(f * 9 + tap) * e.cp[l] + c;
    const long long bo = e.bb[l] + (long long)(tap * e.cin[l] + c) * e.F + f;
    if (e.bf16) {
      wb[fo] = vb;
      if (l > 0) wb[bo] = vb;
    } else {
      e.wp[fo] = v;
      if (l > 0) e.wp[bo] = v;
    }
  }
}

// the update of parameter i with gradient gi (packed copy position from segment s0 when it holds i)
__device__ __forceinline__ void adam_elem(const AdamArgs& A, const PackArgs& pk, long long i, float gi, float bc1,
                                          float bc2, int s0) {
  const float mi = A.b1 * A.m[i] + (1.f - A.b1) * gi;
  const float vi = A.b2 * A.v[i] + (1.f - A.b2) * gi * gi;
  A.m[i] = mi;
  A.v[i] = vi;
  const float pi = A.p[i] - A.lr * (mi / bc1) / (sqrtf(vi / bc2) + A.eps);
  A.p[i] = pi;
  if (A.ep.n && i >= A.ep.lo && i < A.ep.hi) enc_prep_put(A.ep, i, pi);
  float ei = 0.f;
  if (A.ema && i >= A.ema_begin) {
    float* e = A.ema + (i - A.ema_begin);
    ei = A.rho * *e + (1.f - A.rho) * pi;
    *e = ei;
  }
  if (A.shadow) A.shadow[i] = bf16_bits(pi);
  if (pk.n) {
    int critic = 0;
    long long d = -1;
    if (s0 >= 0) {
      const PackSeg& ps = pk.seg[s0];
      const long long loc = i + pk.p_begin - ps.src;
      if (loc >= 0 && loc < (long long)ps.rows * ps.cols) {
        const unsigned r = (unsigned)loc / (unsigned)ps.cols;
        d = ps.dst + (long long)r * ps.ldp + (loc - (long long)r * ps.cols);
        critic = ps.critic;
      }
    }
    if (d < 0) d = pack_pos(pk, i, &critic);
    if (d >= 0) {
      pk.pack[d] = pi;
      if (pk.pack_h) pk.pack_h[d] = bf16_bits(pi);
      if (critic && pk.tpack && A.ema && i >= A.ema_begin) {
        if (pk.tpack32) pk.tpack[d] = ei;
        if (pk.tpack_h) pk.tpack_h[d] = bf16_bits(ei);
      }
    }
  }
}

// Workgroups are dispatched in index order, so the ones with the longest chains
// of dependent loads come first.  With alpha_on, workgroup 0 is the temperature
// step; with fin_on, it ends the update (statistics and counters).  Then one
// workgroup per 64 parameters of every partial-gradient segment: wave w sums the
// partial rows w, w + 4, ... of its lane's parameter, the four wave sums are
// added in wave order (the order colsum() uses), and wave 0 applies the update.
// The rest take 256 * PER consecutive parameters each, skipping the segments.
template <int PER>
__global__ __launch_bounds__(256) void k_adam(AdamArgs A, PackArgs pk, GradSegs gs, int seg_blocks, AlphaJob aj,
                                              int alpha_on, FinishJob fj, int fin_on) {
  int bid = (int)blockIdx.x;
  if (alpha_on || fin_on) {
    if (bid == 0) {
      if (alpha_on) alpha_block(aj, A.lr, A.b1, A.b2, A.eps);
      else finish_block(fj);
      return;
    }
    --bid;
  }
  const float t = (float)(*A.step + 1);
  const float bc1 = 1.f - powf(A.b1, t);
  const float bc2 = 1.f - powf(A.b2, t);
  if (bid < seg_blocks) {
    __shared__ float sh[4][64];
    int b = bid, q = 0;
    while (q < gs.n && b >= (gs.s[q].H + 63) / 64) b -= (gs.s[q++].H + 63) / 64;
    if (q >= gs.n) return;
    const GradSeg& e = gs.s[q];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = b * 64 + lane;
    float sum = 0.f;
    if (j < e.H) {
      const float* pp = e.part + j;
      int r = wave;
      for (; r + 12 < e.nrows; r += 16) {
        float w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = pp[(long long)(r + 4 * k) * e.H];
#pragma unroll
        for (int k = 0; k < 4; ++k) sum += w[k];
      }
      for (; r < e.nrows; r += 4) sum += pp[(long long)r * e.H];
    }
    sh[wave][lane] = sum;
    __syncthreads();
    if (wave == 0 && j < e.H) {
      const float gi = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
      const long long i = e.begin + j;
      gs.gout[i] = gi;
      adam_elem(A, pk, i, gi, bc1, bc2, -1);
    }
    return;
  }
  const long long b0 = (long long)(bid - seg_blocks) * 256 * PER;
  int s0 = -1;
  for (int s = 0; s < pk.n; ++s) {
    const long long loc = b0 + pk.p_begin - pk.seg[s].src;
    if (loc >= 0 && loc < (long long)pk.seg[s].rows * pk.seg[s].cols) { s0 = s; break; }
  }
  // first partial-gradient segment that ends after the workgroup's start (segments sorted by begin)
  int q0 = 0;
  while (q0 < gs.n && gs.s[q0].begin + gs.s[q0].H <= b0) ++q0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const long long i = b0 + u * 256 + threadIdx.x;
    if (i >= A.n) break;
    int q = q0;
    while (q < gs.n && gs.s[q].begin + gs.s[q].H <= i) ++q;
    if (q < gs.n && gs.s[q].begin <= i) continue;   // updated by its segment's workgroup
    adam_elem(A, pk, i, A.g[i], bc1, bc2, s0);
  }
}

int adam(float* p, const float* g, float* m, float* v, long long n, const sq_hparams* hp, const int* step,
         float* ema_target, long long ema_begin, uint16_t* shadow, const PackArgs* pk, hipStream_t st,
         const GradSegs* gs, const AlphaJob* aj, const EncPrepMap* ep, const FinishJob* fj) {
  if (aj && fj) {
    set_error("adam: the temperature step and the update's end cannot share a launch");
    return SQ_EINVAL;
  }
  if (n <= 0 && !aj && !fj) return SQ_OK;
  const int per = (n + 1023) / 1024 >= (long long)kAdamMinPerCU * kAdamCUs ? 4 : 2;
  const long long blocks = n > 0 ? (n + 256 * per - 1) / (256 * per) : 0;
  PackArgs none{};
  GradSegs nogs{};
  AlphaJob noaj{};
  long long seg_blocks = 0;
  if (gs) {
    if (gs->n > 0 && !gs->gout) {
      set_error("adam: partial-gradient segments need a gradient output");
      return SQ_EINVAL;
    }
    for (int i = 0; i < gs->n; ++i) {
      if (i > 0 && gs->s[i].begin < gs->s[i - 1].begin + gs->s[i - 1].H) {
        set_error("adam: partial-gradient segments must be sorted and disjoint");
        return SQ_EINVAL;
      }
      if (gs->s[i].begin < 0 || gs->s[i].begin + gs->s[i].H > n) {
        set_error("adam: partial-gradient segment outside the parameter range");
        return SQ_EINVAL;
      }
      seg_blocks += (gs->s[i].H + 63) / 64;
    }
  }
  const AdamArgs A{p, g, m, v, n, hp->lr, hp->beta1, hp->beta2, hp->adam_eps, step, ema_target, ema_begin, hp->rho,
                   shadow, ep ? *ep : EncPrepMap{}};
  const FinishJob nofj{};
  const unsigned grid = (unsigned)(blocks + seg_blocks + (aj || fj ? 1 : 0));
  if (per == 4)
    k_adam<4><<<grid, 256, 0, st>>>(A, pk ? *pk : none, gs ? *gs : nogs, (int)seg_blocks, aj ? *aj : noaj, aj ? 1 : 0,
                                    fj ? *fj : nofj, fj ? 1 : 0);
  else
    k_adam<2><<<grid, 256, 0, st>>>(A, pk ? *pk : none, gs ? *gs : nogs, (int)seg_blocks, aj ? *aj : noaj, aj ? 1 : 0,
                                    fj ? *fj : nofj, fj ? 1 : 0);
  return launch_status("adam");
}

// the standalone Adam step's counter advance, ordered after the update on its stream
__global__ void k_step_advance(int* step) {
  if (threadIdx.x == 0) *step += 1;
}

int launch_step_advance(int* step, hipStream_t st) {
  k_step_advance<<<1, 64, 0, st>>>(step);
  return launch_status("step advance");
}

// statistics rows of a captured block of updates, copied out to the caller's
// buffer (the last node of the graph; its destination is updated per launch)
__global__ void k_copy_stats(const float* __restrict__ src, float* __restrict__ dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

int launch_copy_stats(const float* src, float* dst, int n, hipStream_t st) {
  k_copy_stats<<<1, 256, 0, st>>>(src, dst, n);
  return launch_status("copy stats");
}

const void* copy_stats_kernel() { return reinterpret_cast<const void*>(&k_copy_stats); }

// rows of every packed segment; padding columns are written as zero
__global__ void k_pack(PackArgs pk, const float* __restrict__ params, const float* __restrict__ target,
                       long long critic_begin) {
  const PackSeg q = pk.seg[blockIdx.y];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)q.rows * q.ldp;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / q.ldp, c = e - r * q.ldp;
    const bool in = c < q.cols;
    const float v = in ? params[q.src + r * q.cols + c] : 0.f;
    pk.pack[q.dst + e] = v;
    if (pk.pack_h) pk.pack_h[q.dst + e] = bf16_bits(v);
    if (q.critic && pk.tpack) {
      const float t = in ? target[q.src - critic_begin + r * q.cols + c] : 0.f;
      pk.tpack[q.dst + e] = t;
      if (pk.tpack_h) pk.tpack_h[q.dst + e] = bf16_bits(t);
    }
  }
}

int pack_weights(const Layout& L, const float* params, const float* target, float* pack, float* tpack,
                 hipStream_t st) {
  PackArgs pk{};
  pk.n = L.n_pack;
  for (int i = 0; i < L.n_pack; ++i) pk.seg[i] = L.pack[i];
  pk.pack = pack;
  pk.tpack = target ? tpack : nullptr;
  pk.pack_h = twin_of(pack, L.pack_total);
  pk.tpack_h = target ? twin_of(tpack, L.pack_critic_end) : nullptr;
  k_pack<<<dim3(64, L.n_pack), 256, 0, st>>>(pk, params, target, L.critic_begin);
  return launch_status("pack_weights");
}

}  // namespace sq
