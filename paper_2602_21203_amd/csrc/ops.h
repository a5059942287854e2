// Host-side composition of the network passes from the kernels: encoder,
// twin critics and actor, forward and backward, plus their workspace plans.
#pragma once

#include "common.h"

namespace sq {

constexpr size_t kSplitFloats = (size_t)4 << 20;   // split-K scratch (16 MB)

struct EncBufs {
  float* h[4];        // post-ReLU conv outputs; h[n_conv-1] is the feature [n][F][s][s]
  float* wprep;       // fused encoder: rearranged conv weights
  float* dh[2];       // ping-pong input gradients
  float* split;       // split-K scratch, kSplitFloats
  float* bias_part;   // conv bias partial sums, 256 * F
  float* enc_part;    // per-workgroup partial gradients of the fused encoder backward
};
void plan_encoder(const Net& net, int n, Bump& b, EncBufs* e, bool with_bwd);
// prepared: e.wprep already holds the rearranged weights of these parameters
// (kept current by the optimiser through an EncPrepMap)
int encoder_forward(const Net& net, int bf16, const float* ep, const Layout& L, const float* x, int n,
                    const EncBufs& e, hipStream_t st, bool prepared = false);
// bfloat16: the minibatch draw sa, the squint of its frames into x (2 sa.B images)
// and the encoder forward in one launch; kNotApplicable when that form does not apply.
// stored: the frames are the block means a ring stored at insertion
int encoder_forward_squint(const Net& net, const float* ep, const Layout& L, const SampleArgs& sa,
                           const uint8_t* obs, const uint8_t* next_obs, float* x, const EncBufs& e, hipStream_t st,
                           bool prepared, bool stored);
// rewrite e.wprep from the parameters (fused path only; no-op otherwise)
int encoder_prepare(const Net& net, int bf16, const float* ep, const Layout& L, const EncBufs& e, hipStream_t st);
// prepared: the fused path's rearranged weights from encoder_forward of the same
// parameters and precision are still in e.wprep (inside one update)
// defer_reduce (fused path only): leave the per-workgroup partial gradients in
// e.enc_part for the optimiser (encoder_grad_seg describes them); dep unused then
int encoder_backward(const Net& net, int bf16, const float* ep, const Layout& L, const float* x, int n,
                     const float* dfeat, const EncBufs& e, float* dep, hipStream_t st,
                     bool prepared = false, bool defer_reduce = false);
// the fused encoder's partial gradients as an optimiser segment (false: no fused path
// in this precision)
bool encoder_grad_seg(const Net& net, int bf16, const Layout& L, const EncBufs& e, int n, GradSeg* seg);
// whether these buffers run the fused encoder in this precision
bool encoder_fused(const Net& net, int bf16, const EncBufs& e);

struct DenseSave { float* xhat; float* rstd; };
struct CriticBufs {
  float* pre;         // [2][n][max(proj, hidden, atoms)]
  float* X1;          // [n][cpad]  = [h | s | a]
  DenseSave t, l1, l2;
  float* g1; float* g2;   // [2][n][hidden]
  float* dA; float* dB;   // [2][n][max(hidden, proj)]
  float* dX1;             // [n][cpad]
  float* part_t; float* part_l1; float* part_l2; float* part_out;
  float* split;
};
// nets = 2 also sizes the forward buffers for critic_forward_pair (online, then target)
void plan_critic(const Net& net, int n, Bump& b, CriticBufs* c, bool with_bwd, int nets = 1);
// cp: base of a critic block (online params + critic_begin, or the target vector);
// cpack: the matching packed weights (nullable: weights are read from cp)
int critic_forward_pair(const Net& net, int bf16, const float* cp, const float* tcp, const float* cpack,
                        const float* tpack, const Layout& L, const float* feat, long long ld_feat, long long sz_feat,
                        const float* s, long long ld_s, long long sz_s, const float* a, const float* ta,
                        long long ld_a, int n, float* logits4, const CriticBufs& c, hipStream_t st,
                        bool trunk_done = false);
// trunk_done: c.X1 already holds the critics' input rows [projection | s | a]
// (trunks_forward, plus the action columns written by the draw and the policy head)
GemmProb critic_trunk_pair_prob(const Net& net, const float* cp, const float* tcp, const float* cpack,
                                const float* tpack, const Layout& L, const float* feat, long long ld_feat,
                                long long sz_feat, int n, const CriticBufs& c);
int critic_forward(const Net& net, int bf16, const float* cp, const float* cpack, const Layout& L, const float* feat,
                   long long ld_feat, const float* s, long long ld_s, const float* a, long long ld_a, int n,
                   float* logits, const CriticBufs& c, hipStream_t st);
// dcp / dfeat / daction nullable; dcp is laid out like the critic block
// out_partials_done: the output-head bias partials of dlogits are already in c.part_out (ce_loss).
// defer_colsum: leave the bias / gain / shift gradients as row-block partials for the optimiser
// (critic_grad_segs / actor_grad_segs describe them).
int critic_backward(const Net& net, int bf16, const float* cp, const float* cpack, const Layout& L, const float* feat,
                    long long ld_feat, const float* dlogits, int n, const CriticBufs& c, float* dcp, float* dfeat,
                    float* daction, hipStream_t st,
                    bool out_partials_done = false, bool defer_colsum = false, const TgBwdJob* tg = nullptr,
                    int ld_dl = 0);   // dlogits rows ld_dl floats apart (0: atoms)
// tg (with daction): also run the policy head's backward on daction (tanh_gauss_bwd
// with tg's arguments); without the critic's own gradients it is the epilogue of
// the product that forms daction, which is then not stored

struct ActorBufs {
  float* pre;          // [n][max(proj, hidden)]
  float* X1;           // [n][apad] = [h | s]
  DenseSave t, l1, l2;
  float* g1; float* g2;  // [n][hidden]
  float* head;         // [n][2A]
  float* save;         // [n][3A]
  float* dA; float* dB;  // [n][max(hidden, proj)]
  float* dX1;          // [n][proj]
  float* dhead;        // [n][ldh], the first 2A columns
  int ldh;
  float* part_t; float* part_l1; float* part_l2; float* part_out;
  float* split;
  // nullable: the sampled actions of rows >= xact_row0 are also written here
  // (row stride ld_xact), straight into a critic's input rows
  float* xact = nullptr; long long ld_xact = 0; int xact_row0 = 0;
};
void plan_actor(const Net& net, int n, Bump& b, ActorBufs* a, bool with_bwd);
// ap: base of the actor block; pack: the whole packed-weight buffer (nullable);
// eps nullable (mean action)
int actor_forward(const Net& net, int bf16, const float* ap, const float* pack, const Layout& L, const float* feat,
                  long long ld_feat, const float* s, long long ld_s, const float* eps, int n, float lo, float hi,
                  float* action, float* logp, const ActorBufs& a, hipStream_t st, bool trunk_done = false);
// trunk_done: a.X1 already holds the actor's input rows [projection | s] (trunks_forward)
GemmProb actor_trunk_prob(const Net& net, const float* ap, const float* pack, const Layout& L, const float* feat,
                          long long ld_feat, int n, const ActorBufs& a);
// The input projections of the update's forward pass and their LayerNorms, each
// pair in one launch: the actor's on the 2B feature rows [s; s'] (a.X1 = [h | s])
// and the online / target critics' on the rows of s / s' (c.X1 = [h | s], the
// action columns being written by others).  They read the same features and do
// not depend on each other.  s: the 2B proprio rows [s; s'], row stride ld_s.
int trunks_forward(const Net& net, int bf16, const float* ap, const float* cp, const float* tcp, const float* pack,
                   const float* cpack, const float* tpack, const Layout& L, const float* feat, long long ld_feat,
                   const float* s, long long ld_s, int B, const ActorBufs& a, const CriticBufs& c, hipStream_t st);
int actor_backward(const Net& net, int bf16, const float* ap, const float* pack, const Layout& L, const float* feat,
                   long long ld_feat, const float* eps, int n, const float* da, long long ld_da, const float* dlogp_vec,
                   const float* dlogp_scalar, float scale, float lo, float hi, const ActorBufs& a, float* dap,
                   hipStream_t st,
                   bool defer_colsum = false, bool dhead_done = false);
// dhead_done: a.dhead and a.part_out already hold the policy head's backward
// (critic_backward with a TgBwdJob); da is then not read

// act(): squint -> encoder -> actor, forward only
struct ActBufs {
  float* x; EncBufs e; ActorBufs a; float* noise;
};
void plan_act(const Net& net, int n, Bump& b, ActBufs* w);
size_t act_bytes_per_obs(const Net& net);

// The partial-gradient segments left by a deferred colsum, relative to the start of
// each optimiser's range (0 for encoder + critic, actor_begin for the actor).
void critic_grad_segs(const Net& net, const Layout& L, const CriticBufs& c, int n, GradSegs* gs);
void actor_grad_segs(const Net& net, const Layout& L, const ActorBufs& a, int n, GradSegs* gs);

}  // namespace sq
