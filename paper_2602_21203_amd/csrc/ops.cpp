// Network passes composed from the kernels (see ops.h).
//
// Linear layers keep torch's layout, W [out, in] row-major, so
//   forward      Y = X W^T + b            gemm(A = X,    B(c, k) = W[c][k])
//   input grad   dX = dY W                gemm(A = dY,   B(c, k) = W[k][c])
//   weight grad  dW = dY^T X              gemm(A(r, k) = dY[k][r], B(c, k) = X[k][c])
// The twin critics run as batch 2 of the same launch (twin parameter blocks
// are a fixed stride apart in the flat vector).
#include "ops.h"
#include "kernels/sample.h"

#include <algorithm>

namespace sq {

// Y = X W^T + b; W rows `ldw` apart (the packed copy pads them), twins `szw` apart,
// biases `szb` apart
static int linear_fwd(int bf16, int n, int out, int in, int batch, const float* X, long long ldx, long long szx,
                      const float* W, long long ldw, long long szw, const float* b, long long szb, float* Y,
                      long long ldy, long long szy, hipStream_t st) {
  MatArg A{X, ldx, 1, szx};
  MatArg Bm{W, ldw, 1, szw};
  OutArg C{Y, ldy, szy, b, szb, 0, 0};
  return gemm(bf16, n, out, in, batch, A, Bm, C, nullptr, 0, st);
}

// where a linear weight is read from: the packed copy when there is one
struct WRef {
  const float* base; const float* pack; long long base_begin;
  const float* W(long long raw, long long packed) const { return pack ? pack + packed : base + (raw - base_begin); }
  long long ld(int in, int ldp) const { return pack ? ldp : in; }
};

static int linear_dw(int bf16, int n, int out, int in, int batch, const float* dY, long long lddy, long long szdy,
                     const float* X, long long ldx, long long szx, float* dW, long long ldw, long long szw,
                     float* split, hipStream_t st) {
  MatArg A{dY, 1, lddy, szdy};
  MatArg Bm{X, 1, ldx, szx};
  OutArg C{dW, ldw, szw, nullptr, 0, 0, 0};
  return gemm(bf16, out, in, n, batch, A, Bm, C, split, split ? kSplitFloats : 0, st);
}

// dX[:, 0:cols] (+)= dY W[:, 0:cols]; W given at its first wanted column, row stride ldw
static int linear_dx(int bf16, int n, int out, int cols, int batch, const float* dY, long long lddy, long long szdy,
                     const float* W, long long ldw, long long szw, float* dX, long long lddx, long long szdx,
                     int accumulate, hipStream_t st) {
  MatArg A{dY, lddy, 1, szdy};
  MatArg Bm{W, 1, ldw, szw};
  OutArg C{dX, lddx, szdx, nullptr, 0, accumulate, 0};
  return gemm(bf16, n, cols, out, batch, A, Bm, C, nullptr, 0, st);
}

// the same products as GemmProb values, for launching a layer's weight and input
// gradients together
static GemmProb prob_dw(int n, int out, int in, int batch, const float* dY, long long lddy, long long szdy,
                        const float* X, long long ldx, long long szx, float* dW, long long ldw, long long szw) {
  return GemmProb{out, in, n, batch, MatArg{dY, 1, lddy, szdy}, MatArg{X, 1, ldx, szx},
                  OutArg{dW, ldw, szw, nullptr, 0, 0, 0}};
}
static GemmProb prob_dx(int n, int out, int cols, int batch, const float* dY, long long lddy, long long szdy,
                        const float* W, long long ldw, long long szw, float* dX, long long lddx, long long szdx) {
  return GemmProb{n, cols, out, batch, MatArg{dY, lddy, 1, szdy}, MatArg{W, 1, ldw, szw},
                  OutArg{dX, lddx, szdx, nullptr, 0, 0, 0}};
}
// input gradient, and the weight gradient when dw is given, in one launch if possible
static int grads(int bf16, const GemmProb& dx, const GemmProb* dw, float* split, hipStream_t st) {
  if (dw) return gemm_pair(bf16, dx, *dw, split, split ? kSplitFloats : 0, st);
  return gemm(bf16, dx.M, dx.N, dx.K, dx.batch, dx.A, dx.B, dx.C, nullptr, 0, st);
}

// ---------------------------------------------------------------- encoder
void plan_encoder(const Net& net, int n, Bump& b, EncBufs* e, bool with_bwd) {
  const sq_dims& d = net.d;
  for (int i = 0; i < 4; ++i) e->h[i] = nullptr;
  if (d.n_conv == 0) {   // state-based: no encoder
    e->dh[0] = e->dh[1] = nullptr;
    e->split = e->bias_part = e->enc_part = e->wprep = nullptr;
    return;
  }
  for (int i = 0; i < d.n_conv; ++i)
    e->h[i] = b.take<float>((size_t)n * d.F * net.conv_side[i] * net.conv_side[i]);
  e->dh[0] = e->dh[1] = nullptr;
  e->split = nullptr;
  e->bias_part = nullptr;
  e->enc_part = nullptr;
  e->wprep = nullptr;
  // the workspace serves both precisions: the fused path's buffers when either has
  // one, the general path's when the FP32 form has none
  if (encoder_fused_ok(d.C, d.F, d.n_conv, net.side, 1)) {
    e->wprep = b.take<float>(encoder_fused_prep_floats(d.C, d.F, d.n_conv));
    if (with_bwd) {
      Layout L;
      make_layout(net, &L);
      e->enc_part = b.take<float>(encoder_fused_part_floats(n, L.enc_end, net.side));
    }
  }
  if (with_bwd && !encoder_fused_ok(d.C, d.F, d.n_conv, net.side, 0)) {
    const size_t big = (size_t)n * d.F * net.conv_side[0] * net.conv_side[0];
    e->dh[0] = b.take<float>(big);
    e->dh[1] = b.take<float>(big);
    e->split = b.take<float>(kSplitFloats);
    e->bias_part = b.take<float>((size_t)256 * d.F);
  }
}

bool encoder_fused(const Net& net, int bf16, const EncBufs& e) {
  const sq_dims& d = net.d;
  return e.wprep && d.n_conv > 0 && encoder_fused_ok(d.C, d.F, d.n_conv, net.side, bf16);
}

int encoder_prepare(const Net& net, int bf16, const float* ep, const Layout& L, const EncBufs& e, hipStream_t st) {
  const sq_dims& d = net.d;
  if (!encoder_fused(net, bf16, e)) return SQ_OK;
  const float* W[4];
  for (int i = 0; i < d.n_conv; ++i) W[i] = ep + L.conv_W[i];
  return encoder_fused_prep(bf16, d.C, d.F, d.n_conv, W, e.wprep, st);
}

int encoder_forward(const Net& net, int bf16, const float* ep, const Layout& L, const float* x, int n,
                    const EncBufs& e, hipStream_t st, bool prepared) {
  const sq_dims& d = net.d;
  if (encoder_fused(net, bf16, e)) {
    const float* b[4];
    float* h[4];
    for (int i = 0; i < d.n_conv; ++i) {
      b[i] = ep + L.conv_b[i];
      h[i] = e.h[i];
    }
    if (!prepared) SQ_TRY(encoder_prepare(net, bf16, ep, L, e, st));
    uint16_t* hh = bf16 ? twin_of(h[d.n_conv - 1], (long long)n * net.flat) : nullptr;
    return encoder_fused_fwd(bf16, d.C, d.F, d.n_conv, net.side, x, n, e.wprep, b, h, st, hh);
  }
  const float* in = x;
  int cin = d.C, hs = net.side;
  for (int i = 0; i < d.n_conv; ++i) {
    SQ_TRY(conv_fwd(bf16, in, n, cin, hs, i ? 1 : 2, ep + L.conv_W[i], ep + L.conv_b[i], d.F, e.h[i], st));
    in = e.h[i];
    cin = d.F;
    hs = net.conv_side[i];
  }
  return SQ_OK;
}

int encoder_forward_squint(const Net& net, const float* ep, const Layout& L, const SampleArgs& sa,
                           const uint8_t* obs, const uint8_t* next_obs, float* x, const EncBufs& e, hipStream_t st,
                           bool prepared, bool stored) {
  const sq_dims& d = net.d;
  if (!encoder_fused(net, 1, e) || d.n_conv != 3) return kNotApplicable;
  const float* b[4];
  float* h[4];
  for (int i = 0; i < d.n_conv; ++i) {
    b[i] = ep + L.conv_b[i];
    h[i] = e.h[i];
  }
  if (!prepared) SQ_TRY(encoder_prepare(net, 1, ep, L, e, st));
  uint16_t* hh = twin_of(h[d.n_conv - 1], (long long)2 * sa.B * net.flat);
  // stored frames are the block means at the squinted side: their squint is k = 1
  return stored ? encoder_fused_fwd_squint(sa, obs, next_obs, net.side, net.side, d.C, d.F, d.n_conv, 1, x, e.wprep,
                                           b, h, hh, st)
                : encoder_fused_fwd_squint(sa, obs, next_obs, d.H, d.W, d.C, d.F, d.n_conv, d.k, x, e.wprep, b, h,
                                           hh, st);
}

bool encoder_grad_seg(const Net& net, int bf16, const Layout& L, const EncBufs& e, int n, GradSeg* seg) {
  if (!e.enc_part || !encoder_fused(net, bf16, e)) return false;
  *seg = GradSeg{L.enc_begin, (int)(L.enc_end - L.enc_begin), encoder_fused_part_rows(n, net.side), e.enc_part};
  return true;
}

int encoder_backward(const Net& net, int bf16, const float* ep, const Layout& L, const float* x, int n,
                     const float* dfeat, const EncBufs& e, float* dep, hipStream_t st,
                     bool prepared, bool defer_reduce) {
  const sq_dims& d = net.d;
  if (e.enc_part && encoder_fused(net, bf16, e)) {
    const float* W[4];
    const float* h[4];
    long long Wo[4], bo[4];
    for (int i = 0; i < d.n_conv; ++i) {
      W[i] = ep + L.conv_W[i];
      h[i] = e.h[i];
      Wo[i] = L.conv_W[i];
      bo[i] = L.conv_b[i];
    }
    if (!prepared) SQ_TRY(encoder_fused_prep(bf16, d.C, d.F, d.n_conv, W, e.wprep, st));
    return encoder_fused_bwd(bf16, d.C, d.F, d.n_conv, net.side, x, n, dfeat, e.wprep, h, Wo, bo, L.enc_end,
                             e.enc_part, defer_reduce ? nullptr : dep, st);
  }
  const float* dh = dfeat;
  for (int i = d.n_conv - 1; i >= 0; --i) {
    const float* in = i ? e.h[i - 1] : x;
    const int cin = i ? d.F : d.C;
    const int hin = i ? net.conv_side[i - 1] : net.side;
    const int hw = net.conv_side[i] * net.conv_side[i];
    SQ_TRY(conv_dw(bf16, in, n, cin, hin, i ? 1 : 2, dh, e.h[i], d.F, dep + L.conv_W[i], e.split, kSplitFloats, st));
    SQ_TRY(conv_bias_grad(dh, e.h[i], n, d.F, hw, dep + L.conv_b[i], e.bias_part, st));
    if (i > 0) {
      float* dx = e.dh[i & 1];
      SQ_TRY(conv_dx(bf16, dh, e.h[i], n, d.F, hin, ep + L.conv_W[i], d.F, dx, st));
      dh = dx;
    }
  }
  return SQ_OK;
}

// ---------------------------------------------------------------- critic
void plan_critic(const Net& net, int n, Bump& b, CriticBufs* c, bool with_bwd, int nets) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, N = d.atoms, cin = net.cpad;
  const int wmax = std::max(std::max(H, P), N);
  const size_t k = (size_t)nets;
  c->pre = b.take<float>(2 * k * n * wmax);
  c->X1 = b.take<float>(k * n * cin);
  c->t.xhat = b.take<float>(k * n * P);
  c->t.rstd = b.take<float>(k * n);
  c->l1.xhat = b.take<float>(2 * k * n * H);
  c->l1.rstd = b.take<float>(2 * k * n);
  c->l2.xhat = b.take<float>(2 * k * n * H);
  c->l2.rstd = b.take<float>(2 * k * n);
  c->g1 = b.take<float>(2 * k * n * H);
  c->g2 = b.take<float>(2 * k * n * H);
  c->dA = c->dB = c->dX1 = c->part_t = c->part_l1 = c->part_l2 = c->part_out = c->split = nullptr;
  if (with_bwd) {
    const int pr = ln_bwd_partial_rows(n);
    const int w = std::max(H, P);
    c->dA = b.take<float>((size_t)2 * n * w);
    c->dB = b.take<float>((size_t)2 * n * w);
    c->dX1 = b.take<float>((size_t)n * cin);
    c->part_t = b.take<float>((size_t)3 * pr * P);
    c->part_l1 = b.take<float>((size_t)2 * 3 * pr * H);
    c->part_l2 = b.take<float>((size_t)2 * 3 * pr * H);
    c->part_out = b.take<float>((size_t)2 * pr * N);
    c->split = b.take<float>(kSplitFloats);
  }
}

int critic_forward(const Net& net, int bf16, const float* cp, const float* cpack, const Layout& L, const float* feat,
                   long long ld_feat, const float* s, long long ld_s, const float* a, long long ld_a, int n,
                   float* logits, const CriticBufs& c, hipStream_t st) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, N = d.atoms, cin = net.cin_critic, cld = net.cpad;
  const long long c0 = L.critic_begin;
  const long long tw = L.q[1].l1.W - L.q[0].l1.W;
  const WRef w{cp, cpack, c0};
  const long long twW = cpack ? L.q[1].l1.Wp - L.q[0].l1.Wp : tw;
  const long long nH = (long long)n * H;
  const Dense& T = L.ctrunk;
  const Twin& q = L.q[0];
  SQ_TRY(linear_fwd(bf16, n, P, net.flat, 1, feat, ld_feat, 0, w.W(T.W, T.Wp), w.ld(T.in, T.ldp), 0,
                    cp + (T.b - c0), 0, c.pre, P, 0, st));
  SQ_TRY(ln_act_fwd(c.pre, P, 0, n, P, 1, cp + (T.g - c0), cp + (T.beta - c0), 0, 1, c.X1, cld, 0, c.t.xhat,
                    c.t.rstd, s, ld_s, d.proprio, a, ld_a, d.action, st));
  SQ_TRY(linear_fwd(bf16, n, H, cin, 2, c.X1, cld, 0, w.W(q.l1.W, q.l1.Wp), w.ld(q.l1.in, q.l1.ldp), twW,
                    cp + (q.l1.b - c0), tw, c.pre, H, nH, st));
  SQ_TRY(ln_act_fwd(c.pre, H, nH, n, H, 2, cp + (q.l1.g - c0), cp + (q.l1.beta - c0), tw, 0, c.g1, H, nH, c.l1.xhat,
                    c.l1.rstd, nullptr, 0, 0, nullptr, 0, 0, st));
  SQ_TRY(linear_fwd(bf16, n, H, H, 2, c.g1, H, nH, w.W(q.l2.W, q.l2.Wp), w.ld(q.l2.in, q.l2.ldp), twW,
                    cp + (q.l2.b - c0), tw, c.pre, H, nH, st));
  SQ_TRY(ln_act_fwd(c.pre, H, nH, n, H, 2, cp + (q.l2.g - c0), cp + (q.l2.beta - c0), tw, 0, c.g2, H, nH, c.l2.xhat,
                    c.l2.rstd, nullptr, 0, 0, nullptr, 0, 0, st));
  return linear_fwd(bf16, n, N, H, 2, c.g2, H, nH, w.W(q.out.W, q.out.Wp), w.ld(q.out.in, q.out.ldp), twW,
                    cp + (q.out.b - c0), tw, logits, N, (long long)n * N, st);
}

// Online (group 0) and target (group 1) twin critics in one pass: the trunk
// runs as a batch of 2 nets, the twin layers as a batch of 4 (online twins, then
// target twins), so every GEMM and LayerNorm launch covers both nets.  Both
// weight sets are read from their packed copies.  logits4 [4][n][atoms].
// the critics' input projections on the features of s (online weights, batch 0)
// and of s' (target weights, batch 1): c.pre [2][n][proj]
GemmProb critic_trunk_pair_prob(const Net& net, const float* cp, const float* tcp, const float* cpack,
                                const float* tpack, const Layout& L, const float* feat, long long ld_feat,
                                long long sz_feat, int n, const CriticBufs& c) {
  const int P = net.d.proj;
  const long long c0 = L.critic_begin;
  const Dense& T = L.ctrunk;
  GemmProb t{n, P, net.flat, 2, MatArg{feat, ld_feat, 1, sz_feat}, MatArg{cpack + T.Wp, T.ldp, 1, 0, tpack + T.Wp, 1},
             OutArg{c.pre, P, (long long)n * P, cp + (T.b - c0), 0, 0, 0, tcp + (T.b - c0), 1}};
  return t;
}

int critic_forward_pair(const Net& net, int bf16, const float* cp, const float* tcp, const float* cpack,
                        const float* tpack, const Layout& L, const float* feat, long long ld_feat, long long sz_feat,
                        const float* s, long long ld_s, long long sz_s, const float* a, const float* ta,
                        long long ld_a, int n, float* logits4, const CriticBufs& c, hipStream_t st, bool trunk_done) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, N = d.atoms, cld = net.cpad;
  const long long c0 = L.critic_begin;
  const long long tw = L.q[1].l1.W - L.q[0].l1.W;
  const long long twW = L.q[1].l1.Wp - L.q[0].l1.Wp;
  const long long nH = (long long)n * H;
  const Dense& T = L.ctrunk;
  const Twin& q = L.q[0];
  if (!trunk_done) {
    const GemmProb t = critic_trunk_pair_prob(net, cp, tcp, cpack, tpack, L, feat, ld_feat, sz_feat, n, c);
    SQ_TRY(gemm(bf16, t.M, t.N, t.K, t.batch, t.A, t.B, t.C, nullptr, 0, st));
    const LnGroups grp{1, tcp + (T.g - c0), tcp + (T.beta - c0), sz_s, ta};
    SQ_TRY(ln_act_fwd(c.pre, P, (long long)n * P, n, P, 2, cp + (T.g - c0), cp + (T.beta - c0), 0, 1, c.X1, cld,
                      (long long)n * cld, c.t.xhat, c.t.rstd, s, ld_s, d.proprio, a, ld_a, d.action, st, &grp));
  }
  auto layer = [&](const Dense& D, const float* X, long long ldx, long long szx, int zdiv, int in, float* Y) -> int {
    MatArg A{X, ldx, 1, szx, nullptr, kNoAlt, zdiv};
    MatArg Bm{cpack + D.Wp, D.ldp, 1, twW, tpack + D.Wp, 2};
    OutArg C{c.pre, H, nH, cp + (D.b - c0), tw, 0, 0, tcp + (D.b - c0), 2};
    SQ_TRY(gemm(bf16, n, H, in, 4, A, Bm, C, nullptr, 0, st));
    const LnGroups grp{2, tcp + (D.g - c0), tcp + (D.beta - c0), 0, nullptr};
    const DenseSave& ln = &D == &q.l1 ? c.l1 : c.l2;
    return ln_act_fwd(c.pre, H, nH, n, H, 4, cp + (D.g - c0), cp + (D.beta - c0), tw, 0, Y, H, nH, ln.xhat, ln.rstd,
                      nullptr, 0, 0, nullptr, 0, 0, st, &grp);
  };
  SQ_TRY(layer(q.l1, c.X1, cld, (long long)n * cld, 2, net.cin_critic, c.g1));
  SQ_TRY(layer(q.l2, c.g1, H, nH, 1, H, c.g2));
  MatArg A{c.g2, H, 1, nH};
  MatArg Bm{cpack + q.out.Wp, q.out.ldp, 1, twW, tpack + q.out.Wp, 2};
  OutArg C{logits4, N, (long long)n * N, cp + (q.out.b - c0), tw, 0, 0, tcp + (q.out.b - c0), 2};
  return gemm(bf16, n, N, H, 4, A, Bm, C, nullptr, 0, st);
}

int critic_backward(const Net& net, int bf16, const float* cp, const float* cpack, const Layout& L, const float* feat,
                    long long ld_feat, const float* dlogits, int n, const CriticBufs& c, float* dcp, float* dfeat,
                    float* daction, hipStream_t st,
                    bool out_partials_done, bool defer_colsum, const TgBwdJob* tg, int ld_dl) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, N = d.atoms, cin = net.cin_critic, cld = net.cpad, A = d.action;
  const long long c0 = L.critic_begin;
  const long long tw = L.q[1].l1.W - L.q[0].l1.W;
  const WRef w{cp, cpack, c0};
  const long long twW = cpack ? L.q[1].l1.Wp - L.q[0].l1.Wp : tw;
  const long long nH = (long long)n * H;
  const Dense& T = L.ctrunk;
  const Twin& q = L.q[0];
  const bool params = dcp != nullptr;
  const bool trunk = params || dfeat != nullptr;
  // output heads
  const long long ldl = ld_dl > 0 ? ld_dl : N, nL = (long long)n * ldl;
  if (params && !out_partials_done) SQ_TRY(col_partials(dlogits, ldl, nL, n, N, 2, c.part_out, st));
  {
    const GemmProb dx = prob_dx(n, N, H, 2, dlogits, ldl, nL, w.W(q.out.W, q.out.Wp), w.ld(q.out.in, q.out.ldp), twW,
                                c.dA, H, nH);
    const GemmProb dw = prob_dw(n, N, H, 2, dlogits, ldl, nL, c.g2, H, nH, dcp + (q.out.W - c0), H, tw);
    SQ_TRY(grads(bf16, dx, params ? &dw : nullptr, c.split, st));
  }
  // second hidden layer
  SQ_TRY(ln_act_bwd(c.dA, H, nH, c.g2, H, nH, c.l2.xhat, c.l2.rstd, cp + (q.l2.g - c0), cp + (q.l2.beta - c0), tw,
                    n, H, 2, 0, c.dB, params ? c.part_l2 : nullptr, st));
  {
    const GemmProb dx = prob_dx(n, H, H, 2, c.dB, H, nH, w.W(q.l2.W, q.l2.Wp), w.ld(q.l2.in, q.l2.ldp), twW, c.dA,
                                H, nH);
    const GemmProb dw = prob_dw(n, H, H, 2, c.dB, H, nH, c.g1, H, nH, dcp + (q.l2.W - c0), H, tw);
    SQ_TRY(grads(bf16, dx, params ? &dw : nullptr, c.split, st));
  }
  // first hidden layer; the shared input [h | s | a] collects the gradient of both
  // twins as one contraction over k = (twin, hidden unit)
  SQ_TRY(ln_act_bwd(c.dA, H, nH, c.g1, H, nH, c.l1.xhat, c.l1.rstd, cp + (q.l1.g - c0), cp + (q.l1.beta - c0), tw,
                    n, H, 2, 0, c.dB, params ? c.part_l1 : nullptr, st));
  const float* W1a = w.W(L.q[0].l1.W, L.q[0].l1.Wp);
  const float* W1b = w.W(L.q[1].l1.W, L.q[1].l1.Wp);
  const long long ld1 = w.ld(q.l1.in, q.l1.ldp);
  const GemmProb dw1 = prob_dw(n, H, cin, 2, c.dB, H, nH, c.X1, cld, 0, dcp + (q.l1.W - c0), cin, tw);
  if (trunk || daction) {
    const int c0col = trunk ? 0 : P + d.proprio;   // without the trunk only the action columns are wanted
    GemmProb dx = prob_dx(n, H, trunk ? cin : A, 1, c.dB, H, 0, W1a + c0col, ld1, 0, trunk ? c.dX1 : daction,
                          trunk ? cld : A, 0);
    if (H % 32 == 0) {
      dx.K = 2 * H;
      dx.A.kp = c.dB + nH;
      dx.A.kalt = H;
      dx.B.kp = W1b + c0col;
      dx.B.kalt = H;
      if (tg && !trunk && !params) {
        // the policy head's backward is the epilogue of the product forming da
        return gemm_tg_bwd(bf16, dx, A, *tg, st);
      }
      SQ_TRY(grads(bf16, dx, params ? &dw1 : nullptr, c.split, st));
    } else {   // twin by twin, the second accumulating
      SQ_TRY(grads(bf16, dx, params ? &dw1 : nullptr, c.split, st));
      GemmProb dxb = dx;
      dxb.A.p = c.dB + nH;
      dxb.B.p = W1b + c0col;
      dxb.C.accumulate = 1;
      SQ_TRY(grads(bf16, dxb, nullptr, c.split, st));
    }
    if (trunk && daction)
      SQ_TRY_HIP(hipMemcpy2DAsync(daction, (size_t)A * 4, c.dX1 + P + d.proprio, (size_t)cld * 4, (size_t)A * 4, n,
                                  hipMemcpyDeviceToDevice, st));
    if (tg && daction)
      SQ_TRY(tanh_gauss_bwd(tg->save, tg->eps, daction, A, tg->dlogp_vec, tg->dlogp_scalar, tg->scale, tg->lo, tg->hi,
                            n, A, tg->dhead, tg->part, st, tg->ldh));
  } else if (params) {
    SQ_TRY(gemm(bf16, dw1.M, dw1.N, dw1.K, dw1.batch, dw1.A, dw1.B, dw1.C, c.split, kSplitFloats, st));
  }
  if (trunk) {
    // (the LayerNorm backward outputs all go to dB, whose bfloat16 copy the products read)
    SQ_TRY(ln_act_bwd(c.dX1, cld, 0, c.X1, cld, 0, c.t.xhat, c.t.rstd, cp + (T.g - c0), cp + (T.beta - c0), 0, n,
                      P, 1, 1, c.dB, params ? c.part_t : nullptr, st));
    const GemmProb dw = prob_dw(n, P, net.flat, 1, c.dB, P, 0, feat, ld_feat, 0, dcp + (T.W - c0), net.flat, 0);
    if (dfeat) {
      const GemmProb dx = prob_dx(n, P, net.flat, 1, c.dB, P, 0, w.W(T.W, T.Wp), w.ld(T.in, T.ldp), 0, dfeat,
                                  net.flat, 0);
      SQ_TRY(grads(bf16, dx, params ? &dw : nullptr, c.split, st));
    } else if (params) {
      SQ_TRY(gemm(bf16, dw.M, dw.N, dw.K, dw.batch, dw.A, dw.B, dw.C, c.split, kSplitFloats, st));
    }
  }
  if (params && !defer_colsum) {
    const int pr = ln_bwd_partial_rows(n);
    ColSegs sg{};
    sg.n = 4;
    sg.s[0] = ColSeg{c.part_out, pr, N, 1, 2, {dcp + (q.out.b - c0), nullptr, nullptr}, tw, 0};
    sg.s[1] = ColSeg{c.part_l2, pr, H, 3, 2, {dcp + (q.l2.b - c0), dcp + (q.l2.g - c0), dcp + (q.l2.beta - c0)}, tw, 0};
    sg.s[2] = ColSeg{c.part_l1, pr, H, 3, 2, {dcp + (q.l1.b - c0), dcp + (q.l1.g - c0), dcp + (q.l1.beta - c0)}, tw, 0};
    sg.s[3] = ColSeg{c.part_t, pr, P, 3, 1, {dcp + (T.b - c0), dcp + (T.g - c0), dcp + (T.beta - c0)}, 0, 0};
    SQ_TRY(colsum(sg, st));
  }
  return SQ_OK;
}

// ---------------------------------------------------------------- actor
void plan_actor(const Net& net, int n, Bump& b, ActorBufs* a, bool with_bwd) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, A = d.action, cin = net.apad;
  const int w = std::max(H, P);
  a->pre = b.take<float>((size_t)n * std::max(w, 2 * A));
  a->X1 = b.take<float>((size_t)n * cin);
  a->t.xhat = b.take<float>((size_t)n * P);
  a->t.rstd = b.take<float>(n);
  a->l1.xhat = b.take<float>((size_t)n * H);
  a->l1.rstd = b.take<float>(n);
  a->l2.xhat = b.take<float>((size_t)n * H);
  a->l2.rstd = b.take<float>(n);
  a->g1 = b.take<float>((size_t)n * H);
  a->g2 = b.take<float>((size_t)n * H);
  a->head = b.take<float>((size_t)n * 2 * A);
  a->save = b.take<float>((size_t)n * 3 * A);
  a->ldh = (2 * A + 7) / 8 * 8;   // dhead rows 16-byte aligned (the products read its bfloat16 copy)
  a->dA = a->dB = a->dX1 = a->dhead = a->part_t = a->part_l1 = a->part_l2 = a->part_out = a->split = nullptr;
  if (with_bwd) {
    const int pr = ln_bwd_partial_rows(n);
    a->dA = b.take<float>((size_t)n * w);
    a->dB = b.take<float>((size_t)n * w);
    a->dX1 = b.take<float>((size_t)n * P);
    a->dhead = b.take<float>((size_t)n * a->ldh);
    a->part_t = b.take<float>((size_t)3 * pr * P);
    a->part_l1 = b.take<float>((size_t)3 * pr * H);
    a->part_l2 = b.take<float>((size_t)3 * pr * H);
    a->part_out = b.take<float>((size_t)pr * 2 * A);
    a->split = b.take<float>(kSplitFloats);
  }
}

// the actor's input projection: a.pre [n][proj]
GemmProb actor_trunk_prob(const Net& net, const float* ap, const float* pack, const Layout& L, const float* feat,
                          long long ld_feat, int n, const ActorBufs& a) {
  const int P = net.d.proj;
  const long long a0 = L.actor_begin;
  const WRef w{ap, pack, a0};
  const Dense& T = L.atrunk;
  GemmProb t{n, P, net.flat, 1, MatArg{feat, ld_feat, 1, 0}, MatArg{w.W(T.W, T.Wp), w.ld(T.in, T.ldp), 1, 0},
             OutArg{a.pre, P, 0, ap + (T.b - a0), 0, 0, 0}};
  return t;
}

int trunks_forward(const Net& net, int bf16, const float* ap, const float* cp, const float* tcp, const float* pack,
                   const float* cpack, const float* tpack, const Layout& L, const float* feat, long long ld_feat,
                   const float* s, long long ld_s, int B, const ActorBufs& a, const CriticBufs& c, hipStream_t st) {
  SQ_TRY(gemm_pair(bf16, actor_trunk_prob(net, ap, pack, L, feat, ld_feat, 2 * B, a),
                   critic_trunk_pair_prob(net, cp, tcp, cpack, tpack, L, feat, ld_feat, (long long)B * ld_feat, B, c),
                   nullptr, 0, st));
  const int P = net.d.proj, S = net.d.proprio;
  const long long a0 = L.actor_begin, c0 = L.critic_begin;
  const Dense& Ta = L.atrunk;
  const Dense& Tc = L.ctrunk;
  const LnFwdJob ja = ln_fwd_job(a.pre, P, 0, 2 * B, P, 1, ap + (Ta.g - a0), ap + (Ta.beta - a0), 0, 1, a.X1,
                                 net.apad, 0, a.t.xhat, a.t.rstd, s, ld_s, S, nullptr, 0, 0);
  const LnGroups grp{1, tcp + (Tc.g - c0), tcp + (Tc.beta - c0), (long long)B * ld_s, nullptr};
  const LnFwdJob jc = ln_fwd_job(c.pre, P, (long long)B * P, B, P, 2, cp + (Tc.g - c0), cp + (Tc.beta - c0), 0, 1,
                                 c.X1, net.cpad, (long long)B * net.cpad, c.t.xhat, c.t.rstd, s, ld_s, S, nullptr, 0,
                                 0, &grp);
  return ln_act_fwd_pair(ja, jc, st);
}

int actor_forward(const Net& net, int bf16, const float* ap, const float* pack, const Layout& L, const float* feat,
                  long long ld_feat, const float* s, long long ld_s, const float* eps, int n, float lo, float hi,
                  float* action, float* logp, const ActorBufs& a, hipStream_t st, bool trunk_done) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, A = d.action, cin = net.cin_actor, ald = net.apad;
  const long long a0 = L.actor_begin;
  const WRef w{ap, pack, a0};
  const Dense& T = L.atrunk;
  if (!trunk_done) {
    const GemmProb t = actor_trunk_prob(net, ap, pack, L, feat, ld_feat, n, a);
    SQ_TRY(gemm(bf16, t.M, t.N, t.K, t.batch, t.A, t.B, t.C, nullptr, 0, st));
    SQ_TRY(ln_act_fwd(a.pre, P, 0, n, P, 1, ap + (T.g - a0), ap + (T.beta - a0), 0, 1, a.X1, ald, 0, a.t.xhat,
                      a.t.rstd, s, ld_s, d.proprio, nullptr, 0, 0, st));
  }
  SQ_TRY(linear_fwd(bf16, n, H, cin, 1, a.X1, ald, 0, w.W(L.al1.W, L.al1.Wp), w.ld(L.al1.in, L.al1.ldp), 0,
                    ap + (L.al1.b - a0), 0, a.pre, H, 0, st));
  SQ_TRY(ln_act_fwd(a.pre, H, 0, n, H, 1, ap + (L.al1.g - a0), ap + (L.al1.beta - a0), 0, 0, a.g1, H, 0, a.l1.xhat,
                    a.l1.rstd, nullptr, 0, 0, nullptr, 0, 0, st));
  SQ_TRY(linear_fwd(bf16, n, H, H, 1, a.g1, H, 0, w.W(L.al2.W, L.al2.Wp), w.ld(L.al2.in, L.al2.ldp), 0,
                    ap + (L.al2.b - a0), 0, a.pre, H, 0, st));
  SQ_TRY(ln_act_fwd(a.pre, H, 0, n, H, 1, ap + (L.al2.g - a0), ap + (L.al2.beta - a0), 0, 0, a.g2, H, 0, a.l2.xhat,
                    a.l2.rstd, nullptr, 0, 0, nullptr, 0, 0, st));
  MatArg X{a.g2, H, 1, 0};
  MatArg Wm{w.W(L.aout.W, L.aout.Wp), w.ld(L.aout.in, L.aout.ldp), 1, 0};
  return gemm_tanh_gauss(bf16, n, A, H, X, Wm, ap + (L.aout.b - a0), eps, lo, hi, action, logp, a.save, a.head, st,
                         a.xact, a.ld_xact, a.xact_row0);
}

int actor_backward(const Net& net, int bf16, const float* ap, const float* pack, const Layout& L, const float* feat,
                   long long ld_feat, const float* eps, int n, const float* da, long long ld_da, const float* dlogp_vec,
                   const float* dlogp_scalar, float scale, float lo, float hi, const ActorBufs& a, float* dap,
                   hipStream_t st,
                   bool defer_colsum, bool dhead_done) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, A = d.action, cin = net.cin_actor, ald = net.apad;
  const long long a0 = L.actor_begin;
  const WRef w{ap, pack, a0};
  const Dense& T = L.atrunk;
  if (!dhead_done)
    SQ_TRY(tanh_gauss_bwd(a.save, eps, da, ld_da, dlogp_vec, dlogp_scalar, scale, lo, hi, n, A, a.dhead, a.part_out,
                          st, a.ldh));
  {
    const GemmProb dx = prob_dx(n, 2 * A, H, 1, a.dhead, a.ldh, 0, w.W(L.aout.W, L.aout.Wp),
                                w.ld(L.aout.in, L.aout.ldp), 0, a.dA, H, 0);
    const GemmProb dw = prob_dw(n, 2 * A, H, 1, a.dhead, a.ldh, 0, a.g2, H, 0, dap + (L.aout.W - a0), H, 0);
    SQ_TRY(grads(bf16, dx, &dw, a.split, st));
  }
  SQ_TRY(ln_act_bwd(a.dA, H, 0, a.g2, H, 0, a.l2.xhat, a.l2.rstd, ap + (L.al2.g - a0), ap + (L.al2.beta - a0), 0, n,
                    H, 1, 0, a.dB, a.part_l2, st));
  {
    const GemmProb dx = prob_dx(n, H, H, 1, a.dB, H, 0, w.W(L.al2.W, L.al2.Wp), w.ld(L.al2.in, L.al2.ldp), 0, a.dA,
                                H, 0);
    const GemmProb dw = prob_dw(n, H, H, 1, a.dB, H, 0, a.g1, H, 0, dap + (L.al2.W - a0), H, 0);
    SQ_TRY(grads(bf16, dx, &dw, a.split, st));
  }
  SQ_TRY(ln_act_bwd(a.dA, H, 0, a.g1, H, 0, a.l1.xhat, a.l1.rstd, ap + (L.al1.g - a0), ap + (L.al1.beta - a0), 0, n,
                    H, 1, 0, a.dB, a.part_l1, st));
  {
    // only the projection columns of the actor input need a gradient
    const GemmProb dx = prob_dx(n, H, P, 1, a.dB, H, 0, w.W(L.al1.W, L.al1.Wp), w.ld(L.al1.in, L.al1.ldp), 0,
                                a.dX1, P, 0);
    const GemmProb dw = prob_dw(n, H, cin, 1, a.dB, H, 0, a.X1, ald, 0, dap + (L.al1.W - a0), cin, 0);
    SQ_TRY(grads(bf16, dx, &dw, a.split, st));
  }
  SQ_TRY(ln_act_bwd(a.dX1, P, 0, a.X1, ald, 0, a.t.xhat, a.t.rstd, ap + (T.g - a0), ap + (T.beta - a0), 0, n, P, 1,
                    1, a.dB, a.part_t, st));
  SQ_TRY(linear_dw(bf16, n, P, net.flat, 1, a.dB, P, 0, feat, ld_feat, 0, dap + (T.W - a0), net.flat, 0, a.split, st));
  if (defer_colsum) return SQ_OK;
  const int pr = ln_bwd_partial_rows(n);
  ColSegs sg{};
  sg.n = 4;
  sg.s[0] = ColSeg{a.part_out, tanh_gauss_partial_rows(n), 2 * A, 1, 1, {dap + (L.aout.b - a0), nullptr, nullptr},
                   0, 0};
  sg.s[1] = ColSeg{a.part_l2, pr, H, 3, 1, {dap + (L.al2.b - a0), dap + (L.al2.g - a0), dap + (L.al2.beta - a0)}, 0, 0};
  sg.s[2] = ColSeg{a.part_l1, pr, H, 3, 1, {dap + (L.al1.b - a0), dap + (L.al1.g - a0), dap + (L.al1.beta - a0)}, 0, 0};
  sg.s[3] = ColSeg{a.part_t, pr, P, 3, 1, {dap + (T.b - a0), dap + (T.g - a0), dap + (T.beta - a0)}, 0, 0};
  return colsum(sg, st);
}

static void sort_segs(GradSegs* gs) {
  std::sort(gs->s, gs->s + gs->n, [](const GradSeg& x, const GradSeg& y) { return x.begin < y.begin; });
}

void critic_grad_segs(const Net& net, const Layout& L, const CriticBufs& c, int n, GradSegs* gs) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj, N = d.atoms;
  const int pr = ln_bwd_partial_rows(n);
  gs->n = 0;
  auto add = [&](long long begin, int width, const float* part) { gs->s[gs->n++] = GradSeg{begin, width, pr, part}; };
  for (int t = 0; t < 2; ++t) {
    const Twin& q = L.q[t];
    add(q.out.b, N, c.part_out + (size_t)t * pr * N);
    const long long l2[3] = {q.l2.b, q.l2.g, q.l2.beta}, l1[3] = {q.l1.b, q.l1.g, q.l1.beta};
    for (int k = 0; k < 3; ++k) {
      add(l2[k], H, c.part_l2 + (size_t)(t * 3 + k) * pr * H);
      add(l1[k], H, c.part_l1 + (size_t)(t * 3 + k) * pr * H);
    }
  }
  const long long tr[3] = {L.ctrunk.b, L.ctrunk.g, L.ctrunk.beta};
  for (int k = 0; k < 3; ++k) add(tr[k], P, c.part_t + (size_t)k * pr * P);
  sort_segs(gs);
}

void actor_grad_segs(const Net& net, const Layout& L, const ActorBufs& a, int n, GradSegs* gs) {
  const sq_dims& d = net.d;
  const int H = d.hidden, P = d.proj;
  const int pr = ln_bwd_partial_rows(n);
  const long long a0 = L.actor_begin;
  gs->n = 0;
  gs->s[gs->n++] = GradSeg{L.aout.b - a0, 2 * d.action, tanh_gauss_partial_rows(n), a.part_out};
  const long long l2[3] = {L.al2.b, L.al2.g, L.al2.beta}, l1[3] = {L.al1.b, L.al1.g, L.al1.beta};
  const long long tr[3] = {L.atrunk.b, L.atrunk.g, L.atrunk.beta};
  for (int k = 0; k < 3; ++k) {
    gs->s[gs->n++] = GradSeg{l2[k] - a0, H, pr, a.part_l2 + (size_t)k * pr * H};
    gs->s[gs->n++] = GradSeg{l1[k] - a0, H, pr, a.part_l1 + (size_t)k * pr * H};
    gs->s[gs->n++] = GradSeg{tr[k] - a0, P, pr, a.part_t + (size_t)k * pr * P};
  }
  sort_segs(gs);
}

}  // namespace sq
