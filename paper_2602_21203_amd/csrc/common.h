// Internal declarations shared by the HIP kernels and the host orchestration.
// Not part of the public C ABI (that is include/squint.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "squint.h"

namespace sq {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
#define SQ_TRY_HIP(expr)                                                        \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess) {                                                     \
      ::sq::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),    \
                      __FILE__, __LINE__);                                      \
      return SQ_EDEVICE;                                                        \
    }                                                                           \
  } while (0)
#define SQ_TRY(expr)            \
  do {                          \
    int _s = (expr);            \
    if (_s != SQ_OK) return _s; \
  } while (0)

inline int launch_status(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("launch of %s failed: %s", what, hipGetErrorString(e));
    return SQ_EDEVICE;
  }
  return SQ_OK;
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// returned by a launcher whose fused or specialised form does not apply to its
// arguments (nothing enqueued; the caller takes the general path)
constexpr int kNotApplicable = -1;

// ------------------------------------------------------------------ derived dims
struct Net {
  sq_dims d;
  int side;            // squinted side (16)
  int conv_side[4];    // output side of each conv
  int flat;            // encoder feature width
  int cin_critic;      // proj + proprio + action
  int cin_actor;       // proj + proprio
  int cpad, apad;      // their row strides in workspace buffers (multiples of 8)
  int img;             // C * side * side (one squinted image)
};
int make_net(const sq_dims* d, Net* n);   // validates; SQ_EINVAL on bad dims

// canonical flat parameter layout (offsets in floats).  Wp / ldp: the weight's
// place in the packed copy (rows padded to a multiple of 8 floats, every
// tensor 64-float aligned) that the vector GEMM path reads.
struct Dense { long long W, b, g, beta; int out, in; long long Wp; int ldp; };
struct Head { long long W, b; int out, in; long long Wp; int ldp; };
struct Twin { Dense l1, l2; Head out; };
struct PackSeg { long long src, dst; int rows, cols, ldp, critic; };
struct Layout {
  long long conv_W[4], conv_b[4];
  Dense ctrunk; Twin q[2];
  Dense atrunk; Dense al1, al2; Head aout;
  long long log_alpha;
  long long enc_begin, enc_end, critic_begin, critic_end, actor_begin, actor_end, total;
  int n_tensors;
  long long tensor_off[64];
  // packed linear weights: critic block first ([0, pack_critic_end), also the
  // layout of the target critic's pack), then the actor block
  int n_pack;
  PackSeg pack[16];
  long long pack_critic_end, pack_total;
};
void make_layout(const Net& n, Layout* L);

// ------------------------------------------------------------------ bump allocator
struct Bump {
  char* base;     // nullptr while measuring
  size_t off = 0;
  template <class T> T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct EncPrepMap;   // (defined with the optimiser's arguments below)

// ------------------------------------------------------------------ kernel launchers
// Every launcher enqueues on `st` and returns SQ_OK or SQ_EDEVICE.

// counters layout (int32 device array)
enum { CTR_U = 0, CTR_TC = 1, CTR_TA = 2, CTR_TALPHA = 3, CTR_N = 4 };

// rng.hip
// the update's minibatch draw (kernels/sample.h); dev_size (nullable): the
// replay's row count read on the device (growing ring)
struct SampleArgs;
SampleArgs sample_args(unsigned long long seed, const int* ctr, int size, const int* dev_size, int B, int A, int S,
                       const float* proprio, const float* next_proprio, const float* action, const float* reward,
                       const uint8_t* done, int* idx, float* eps2B, float* S2, float* Arep, long long ld_arep,
                       float* r, float* d);
int launch_sample_batch(const SampleArgs& s, hipStream_t st);
// the draw and the squint of the sampled obs / next_obs rows in one launch (the
// squint workgroups compute their rows' indices themselves); falls back to two
// launches where the fused squint kernel does not apply
int launch_sample_squint(const SampleArgs& s, const uint8_t* obs, const uint8_t* next_obs, int H, int W, int C,
                         int k, float* out, hipStream_t st);
int launch_indices(unsigned long long seed, unsigned update, int size, int n, int* idx, hipStream_t st);
int launch_gaussian(unsigned long long seed, unsigned update, unsigned stream_id, int n, float* out,
                    hipStream_t st);
int launch_act_noise(unsigned long long seed, unsigned long long request_id, int rows, int A, float* out,
                     hipStream_t st);

// squint.hip: frames [*, H, W, C] uint8, rows idx (nullable) -> out [n, C, side, side]
int squint_ok(int H, int W, int C, int k);
int launch_squint(const uint8_t* frames, const int* idx, int n, int H, int W, int C, int k, int bf16_out,
                  void* out, long long out_row_stride, hipStream_t st);
// 2B images: obs rows idx[0..B) then next_obs rows idx[0..B)
int launch_squint_pair(const uint8_t* obs, const uint8_t* next_obs, const int* idx, int B, int H, int W,
                       int C, int k, float* out, hipStream_t st);

// serving: frames gathered through per-row pointers
int launch_squint_rows(const uint8_t* const* rows, int n, int H, int W, int C, int k, float* out, hipStream_t st);
// the small fields of the transitions a squint-at-insertion launch stores, and
// the ring's device counters {pos, size} after the insertion
struct RingRows {
  const float *proprio, *next_proprio, *action, *reward;
  const uint8_t* done;
  float *r_proprio, *r_next, *r_action, *r_reward;
  uint8_t* r_done;
  int P, A;
  int* ctr;
  int new_pos, new_size;
};
// env.hip: the synthetic environment stub's device state (n environments)
struct EnvState {
  int n, H, W, C, P, A, T;
  unsigned k0, k1;
  float* s;       // [n, P] proprio
  float* g;       // [n, 2] goal
  int* t;         // [n] step within the episode
  int* ep;        // [n] episode number
  int* stack;     // [n, 3, 2] pixel positions of the frame stack, newest first
};
int env_reset_all(const EnvState& E, uint8_t* obs, hipStream_t st);
// prop_t receives the pre-step proprio; obs_next the observation of the next step
int env_step(const EnvState& E, const float* action, float* prop_t, uint8_t* next_obs, float* next_prop,
             float* reward, uint8_t* done, uint8_t* obs_next, hipStream_t st);
// where a squint launch writes (see squint.hip)
enum { kSqF32 = 0, kSqBF16 = 1, kSqU8 = 2 };
struct SqDst { int mode; void* out; void* out1; long long row_stride; int pos, cap; RingRows f; };
// Workgroup order of the linear-layer products: consecutive workgroup ids go to
// the eight XCDs in turn, each with its own L2, so the linear id b of a
// gx x gy x gz grid is remapped (when the tile count is a multiple of 8) to give
// every XCD a contiguous run of tiles, in groups of 8 row tiles -- about an 8 x 8
// block of output tiles per XCD.  A bijection onto the tiles for any grid.
__host__ __device__ __forceinline__ void tile_of(int b, int gx, int gy, int gz, int& bx, int& by, int& bz) {
  const int T = gx * gy * gz;
  if (T % 8 == 0) b = (b % 8) * (T / 8) + b / 8;
  const int per = gx * gy;
  bz = b / per;
  const int p = b - bz * per;
  constexpr int GM = 8;
  const int grp = p / (GM * gy), first = grp * GM;
  const int gm = gx - first < GM ? gx - first : GM;
  const int q = p - grp * GM * gy;
  bx = first + q % gm;
  by = q / gm;
}
// ring row of the i-th transition of an insertion at write position pos: (pos + i)
// mod cap in 64-bit arithmetic (pos + i can pass 2^31 when cap is near 2^31 - 1)
__host__ __device__ __forceinline__ int ring_row(int pos, long long i, int cap) {
  return (int)(((long long)pos + i) % (long long)cap);
}
// squint at insertion: n transitions' obs and next_obs [n, H, W, C] -> uint8 block
// means [side, side, C] in rows (pos + i) % cap of ring_obs / ring_next, and the
// transitions' small fields into the same rows (f)
int launch_squint_insert(const uint8_t* obs, const uint8_t* next_obs, int n, int H, int W, int C, int k,
                         uint8_t* ring_obs, uint8_t* ring_next, int pos, int cap, const RingRows& f,
                         hipStream_t st);
// serve.hip: per-row gather / scatter of small vectors, per-row act noise
int gather_rows(const float* const* src, int width, int n, float* dst, hipStream_t st);
int scatter_rows(const float* src, int width, int n, float* const* dst, hipStream_t st);
int act_noise_rows(unsigned long long seed, const unsigned long long* ids, const int* rows, const int* sample, int n,
                   int A, float* eps, hipStream_t st);

// gemm.hip
// Batch index z of an operand: zi = z / zdiv; element (r, k) at
// p[zi*sz + r*lr + k*lk] for zi < zalt, else alt[(zi - zalt)*sz + r*lr + k*lk]
// (two groups of batches in separate allocations, e.g. online and target nets).
constexpr int kNoAlt = 1 << 30;
// k >= kalt (a multiple of 32): element (r, k) read from kp as (r, k - kalt), with
// the same strides -- a contraction over two blocks laid end to end along k.
struct MatArg {
  const float* p; long long lr, lk, sz;
  const float* alt = nullptr; int zalt = kNoAlt; int zdiv = 1;
  const float* kp = nullptr; int kalt = kNoAlt;
};
struct OutArg {            // C(r, c) at p[z*sz + r*ld + c]
  float* p; long long ld, sz;
  const float* bias; long long bias_sz;  // bias[c] (+ z*bias_sz), nullable
  int accumulate;                        // C += result
  int relu;                              // C = max(C, 0) after bias / accumulate
  const float* bias_alt = nullptr;       // bias of batches z >= bias_zalt: bias_alt + (z - bias_zalt)*bias_sz
  int bias_zalt = kNoAlt;
};
// C(r, c) = sum_k A(r, k) * B(c, k)   (B is addressed by output column, then k).
// scratch (nullable) enables a deterministic split over K for small outputs.
int gemm(int bf16, int M, int N, int K, int batch, MatArg A, MatArg B, OutArg C, float* scratch,
         size_t scratch_floats, hipStream_t st);
// C = A B^T (+ bias) on bfloat16-stored operands, A(r, k) = A[z a_sz + r a_lr + k a_lk]
// with a_lk == 1 or a_lr == 1 (B likewise): the product the bfloat16 mode runs when
// both operands have copies
int gemm_bf16_stored(int M, int N, int K, int batch, const uint16_t* A, long long a_lr, long long a_lk,
                     long long a_sz, const uint16_t* B, long long b_lr, long long b_lk, long long b_sz, OutArg C,
                     hipStream_t st);
// twins.cpp: bfloat16 copies ("twins") of FP32 operand buffers, written by the
// buffers' producers and read by the products in the bfloat16 mode
int twins_enabled();
int set_twins_enabled(int on);
void twin_register(const void* owner, const float* f, long long n, uint16_t* h);
void twin_unregister(const void* owner);
// the twin of [f, f + n), or nullptr when no registered buffer holds that range
uint16_t* twin_of(const float* f, long long n = 1);
// FP32 values no longer kept: [f, f + n)'s producers write the twin only (owner's
// registration); fp32_dropped(p) tells whether p lies in such a range
void fp32_drop_register(const void* owner, const float* f, long long n);
bool fp32_dropped(const float* f);
// products enqueued on twins so far (process-wide)
void note_copy_product();
long long copy_products();
// policy head [n][2A] = X W^T + bias with the tanh-Gaussian sample (eps given) or the
// mean action (eps null) applied per row in the same launch; head is also stored.
// xact (nullable): the actions of rows r >= xact_row0 are also written to
// xact + (r - xact_row0) * ld_xact (a critic's input rows)
int gemm_tanh_gauss(int bf16, int n, int A, int K, MatArg X, MatArg W, const float* bias, const float* eps, float lo,
                    float hi, float* action, float* logp, float* save, float* head, hipStream_t st,
                    float* xact = nullptr, long long ld_xact = 0, int xact_row0 = 0);
struct GemmProb {
  int M, N, K, batch; MatArg A, B; OutArg C;
};
// two independent products; one launch when their operand kinds allow it
int gemm_pair(int bf16, const GemmProb& p0, const GemmProb& p1, float* scratch, size_t scratch_floats,
              hipStream_t st);
// convolutions (3x3 valid, NCHW, W [F, Cin, 3, 3]) as implicit GEMMs
int conv_fwd(int bf16, const float* x, int n, int Cin, int H, int stride, const float* W, const float* b,
             int F, float* out, hipStream_t st);
size_t conv_dw_scratch_floats(int n, int Cin, int H, int stride, int F);
// weight gradient of a conv whose (post-ReLU) output is `out`, upstream grad `dout`
int conv_dw(int bf16, const float* x, int n, int Cin, int H, int stride, const float* dout, const float* out,
            int F, float* dW, float* part, size_t part_floats, hipStream_t st);
// input gradient of a stride-1 conv, through its ReLU
int conv_dx(int bf16, const float* dout, const float* out, int n, int Cin, int H, const float* W, int F,
            float* dx, hipStream_t st);

// encoder.hip: fused encoder for the (C, F, n_conv, side) shapes it is built for.
// The conv weights W[l] are first rewritten by encoder_fused_prep into wp
// (encoder_fused_prep_floats floats, bfloat16-rounded in that form); the fused
// passes read the weights from wp and the biases from b.  Inner activations h[l]
// (l < n_conv - 1) are [n][pixel][F]; the last one is NCHW (the feature vector).
// fused path for these dims in this precision (16 x 16: both; 32 x 32: bfloat16 form)
bool encoder_fused_ok(int C, int F, int n_conv, int side, int bf16);
size_t encoder_fused_part_floats(int n, long long enc_total, int side);
// partial-gradient rows the fused backward writes for n images ([rows][enc_total],
// summed in row order as a GradSeg would); grad == nullptr leaves them unsummed
int encoder_fused_part_rows(int n, int side);
// the prepared-copy map of the fused encoder (false when the geometry has no fused path
// in this precision); W: flat offsets of the conv weights
bool encoder_fused_prep_map(int C, int F, int n_conv, int side, const long long* W, float* wp, int bf16,
                            EncPrepMap* m);
size_t encoder_fused_prep_floats(int C, int F, int n_conv);
int encoder_fused_prep(int bf16, int C, int F, int n_conv, const float* const* W, float* wp, hipStream_t st);
// The minibatch draw, the squint of its obs / next_obs frames (x: FP32 [2B][C][side][side] written for
// the backward) and the bfloat16 encoder forward in one launch; kNotApplicable when the geometry has
// no such form
int encoder_fused_fwd_squint(const SampleArgs& sa, const uint8_t* obs, const uint8_t* next_obs, int H, int W, int C,
                             int F, int n_conv, int k, float* x, const float* wp, const float* const* b,
                             float* const* h, uint16_t* hh, hipStream_t st);
// hh (nullable, bfloat16 form only): the last layer's output is also written there rounded to bfloat16
int encoder_fused_fwd(int bf16, int C, int F, int n_conv, int side, const float* x, int n, const float* wp,
                      const float* const* b, float* const* h, hipStream_t st, uint16_t* hh = nullptr);
// partial gradients of every workgroup in part, their ordered sum in grad[0, total)
int encoder_fused_bwd(int bf16, int C, int F, int n_conv, int side, const float* x, int n, const float* dfeat,
                      const float* wp, const float* const* h, const long long* Woff, const long long* boff,
                      long long total, float* part, float* grad, hipStream_t st);

// rowops.hip
// Second parameter group of a LayerNorm batch (batches z >= zalt read their gain
// and shift from g_alt / beta_alt, their second extra block from e2_alt), and the
// batch stride of the first extra block.
// Batches z >= zalt take the alternative (target-critic) gain and shift; no
// backward runs through them, so their x-hat and rstd are not stored unless
// save_alt is set.
struct LnGroups {
  int zalt; const float* g_alt; const float* beta_alt; long long sz_e1; const float* e2_alt;
  int save_alt = 0;
};
int ln_act_fwd(const float* pre, long long ld_pre, long long sz_pre, int rows, int H, int batch,
               const float* g, const float* beta, long long sz_par, int act_tanh,
               float* y, long long ld_y, long long sz_y, float* xhat, float* rstd,
               const float* e1, long long ld_e1, int w1, const float* e2, long long ld_e2, int w2,
               hipStream_t st, const struct LnGroups* grp = nullptr);
// One LayerNorm forward problem (the arguments of ln_act_fwd), and two problems of
// the same width in one launch (two launches when they cannot share one).
struct LnFwdJob {
  const float* pre; long long ld_pre, sz_pre; int rows, H, batch;
  const float* g; const float* beta; long long sz_par; int act_tanh;
  float* y; long long ld_y, sz_y; float* xhat; float* rstd;
  const float* e1; long long ld_e1; int w1; const float* e2; long long ld_e2; int w2;
  LnGroups grp;
  uint16_t* yh;   // bfloat16 copy of y (nullable; ln_fwd_job fills it)
  int y32;        // y stored in FP32 too (ln_fwd_job: unless its buffer's FP32 values were dropped)
};
LnFwdJob ln_fwd_job(const float* pre, long long ld_pre, long long sz_pre, int rows, int H, int batch, const float* g,
                    const float* beta, long long sz_par, int act_tanh, float* y, long long ld_y, long long sz_y,
                    float* xhat, float* rstd, const float* e1, long long ld_e1, int w1, const float* e2,
                    long long ld_e2, int w2, const LnGroups* grp = nullptr);
int ln_act_fwd_pair(const LnFwdJob& j0, const LnFwdJob& j1, hipStream_t st);
int ln_bwd_partial_rows(int rows);
// y: the forward's output (read for tanh only); beta: the shift (read for ReLU,
// whose mask is recomputed from x-hat, gain and shift); g and beta sz_par apart
int ln_act_bwd(const float* dy, long long ld_dy, long long sz_dy, const float* y, long long ld_y,
               long long sz_y, const float* xhat, const float* rstd, const float* g, const float* beta,
               long long sz_par, int rows, int H, int batch, int act_tanh, float* dpre, float* partials,
               hipStream_t st);
int col_partials(const float* src, long long ld, long long sz, int rows, int N, int batch, float* part,
                 hipStream_t st);
// column sums of partial rows: part [batch][k][nrows][H] -> out[kk][z*out_sz + c]
struct ColSeg {
  const float* part; int nrows, H, k, batch;
  float* out[3]; long long out_sz;
  long long count;   // workgroups, filled by colsum()
};
struct ColSegs { int n; ColSeg s[12]; };
int colsum(ColSegs segs, hipStream_t st);

int tanh_gauss_fwd(const float* head, int rows, int A, const float* eps, float lo, float hi, float* action,
                   float* logp, float* save, hipStream_t st);
// part (nullable): column sums of dhead per block of tanh_gauss_partial_rows rows
int tanh_gauss_partial_rows(int rows);
// dhead rows ldh floats apart (0: 2A)
int tanh_gauss_bwd(const float* save, const float* eps, const float* da, long long ld_da, const float* dlogp_vec,
                   const float* dlogp_scalar, float scale, float lo, float hi, int rows, int A, float* dhead,
                   float* part, hipStream_t st, int ldh = 0);
int mean_action(const float* head, int rows, int A, float* action, hipStream_t st);
// The arguments of tanh_gauss_bwd other than da: the policy head's backward as
// the epilogue of the product that forms da (gemm_tg_bwd)
struct TgBwdJob {
  const float* save; const float* eps; const float* dlogp_vec; const float* dlogp_scalar; float scale, lo, hi;
  float* dhead; float* part;
  int ldh = 0;   // dhead's row stride (0: 2A)
};
struct GemmProb;
// da = dx's product ([rows][A], A <= 32 columns), then tanh_gauss_bwd on it in the
// same launch (dx.C is not written); two launches when the product's shape or
// operands do not allow that
int gemm_tg_bwd(int bf16, const GemmProb& dx, int A, const TgBwdJob& tg, hipStream_t st);

int c51_project_raw(const float* p, const float* reward, const uint8_t* done, const float* bonus,
                    float gamma, int B, int N, float v_min, float v_max, float* m, hipStream_t st);
// Per row of the batch: the C51 projection m of the averaged target-twin softmax
// (bonus -alpha log pi'), tgt_row = E_m[z], then each online twin's cross entropy
// to m: loss_row, dlogits = (softmax - m) / B, q_row = E[z], and (part, nullable)
// the head-bias column partials.  logits4 = [online twins | target twins] [4][B][N].
// cdq: the target twin with the smaller expected value supplies the distribution
// (clipped double-Q) instead of the twin average.
// (dlogits2 rows ld_dl floats apart, 0: N; the bfloat16 copy is written when the buffer has one)
int target_ce(const float* logits4, int B, int N, float v_min, float v_max, const float* reward, const float* done,
              const float* logp_next, const float* log_alpha, float gamma, int cdq, float* m, float* tgt_row,
              float* dlogits2, float* loss_row, float* q_row, float* part, hipStream_t st, int ld_dl = 0);
// The same for a scalar critic (N = 1, Eqs. (1)-(2)): squared error to
// y = r + gamma (1 - d)(Qbar - alpha log pi').
int target_mse(const float* logits4, int B, const float* reward, const float* done, const float* logp_next,
               const float* log_alpha, float gamma, int cdq, float* tgt_row, float* dlogits2, float* loss_row,
               float* q_row, float* part, hipStream_t st);
// actor-loss head of a scalar critic: qa_row = (Q_1 + Q_2) / 2, dq2 = -1 / (2B)
int expected_q_scalar(const float* q2, int B, float* dq2, float* qa_row, hipStream_t st);
int expected_q_grad(const float* logits2, int B, int N, float v_min, float v_max, float* dlogits2,
                    float* qa_row, hipStream_t st, int ld_dl = 0);
int finish_update(const float* loss_row, const float* q_row, const float* tgt_row, const float* logp,
                  const float* qa_row, const float* scal, int B, int actor_step, int* ctr, float* stats,
                  hipStream_t st);
// part: conv_bias_chunks(n, HW) * F floats of scratch
int conv_bias_chunks(int n, int HW);
int conv_bias_grad(const float* dout, const float* out, int n, int F, int HW, float* db, float* part,
                   hipStream_t st);

// adam.hip: step t = *step + 1 (not modified); EMA over i >= ema_begin.
// Packed weight copies (nullable): segments of `pk` whose src lies in
// [p_begin, p_begin + n) are refreshed in `pack` with the new parameters and,
// for critic segments, in `tpack` with the new target values.
struct PackArgs {
  int n; PackSeg seg[16];
  float* pack; float* tpack; long long p_begin;
  uint16_t* pack_h = nullptr; uint16_t* tpack_h = nullptr;   // their bfloat16 copies (nullable)
  int tpack32 = 1;   // 0: the optimiser refreshes only tpack's bfloat16 copy (its FP32 values are not kept)
};
// Gradients that are still row-block partials: parameter i in [begin, begin + H)
// (relative to the optimiser's range) has gradient sum_{r < nrows} part[r * H + i - begin],
// summed in r order (the same sum colsum() forms); the optimiser forms it and
// stores it at gout[i] (the writable gradient vector of the range).
struct GradSeg { long long begin; int H, nrows; const float* part; };
struct GradSegs { int n; GradSeg s[20]; float* gout; };
// Where the encoder's conv weights sit in the fused encoder's prepared copy: per
// layer the forward order [f][tap][CP] at fb and, above the first layer, the
// input-gradient order [tap][c][f] at bb (values rounded to bfloat16 when bf16).
// An Adam launch given this map rewrites the prepared copy with every conv weight
// it updates, so the copy never needs a separate preparation launch.
struct EncPrepMap {
  float* wp; int n, F, bf16;
  long long lo, hi;   // flat range of the conv weights (relative to the optimiser's range)
  long long W[4]; int cin[4], cp[4]; long long fb[4], bb[4];
};
// The temperature step (Alg. 1), run by one extra workgroup of an Adam launch.
// scal receives [0] alpha before, [1] alpha after, [2] alpha loss, [3] mean(-log pi).
// step_snap (nullable): also records ctr[CTR_TA] there, the step count of the
// actor's Adam launch that follows (which may then end the update itself)
struct AlphaJob {
  const float* logp; int B; float target_entropy;
  float* log_alpha; float* grad; float* m; float* v; const int* ctr; float* scal;
  int* step_snap;
};
// *step += 1 in a one-thread launch (the standalone Adam step's counter)
int launch_step_advance(int* step, hipStream_t st);
// dst[0, n) = src[0, n) in one workgroup; copy_stats_kernel() names its kernel
int launch_copy_stats(const float* src, float* dst, int n, hipStream_t st);
const void* copy_stats_kernel();
struct FinishJob;
// fj: one more workgroup of the launch ends the update (statistics, counter
// advance); `step` must then not be one of the counters it advances
int adam(float* p, const float* g, float* m, float* v, long long n, const sq_hparams* hp, const int* step,
         float* ema_target, long long ema_begin, uint16_t* shadow, const PackArgs* pk, hipStream_t st,
         const GradSegs* gs = nullptr, const AlphaJob* aj = nullptr, const EncPrepMap* ep = nullptr,
         const FinishJob* fj = nullptr);
// copy the linear weights of `params` (and the critic block of `target`) into packs
int pack_weights(const Layout& L, const float* params, const float* target, float* pack, float* tpack,
                 hipStream_t st);

}  // namespace sq
