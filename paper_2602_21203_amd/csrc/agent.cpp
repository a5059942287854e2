// The SAC agent: workspace of the fused update, the per-update kernel sequence,
// HIP-graph capture of a block of updates, and the act() policy query.
//
// Per update (Alg. 1 inner loop):
//   sample batch (Philox indices, gather small replay fields, policy noise)
//   squint obs + next_obs -> encoder on 2B images (one pass, current encoder)
//   actor on all 2B rows (next half: target action and log pi; first half:
//     the sample used by the temperature and actor losses)
//   target twin critics on the next half -> averaged softmax -> C51 projection
//   online twin critics on the first half -> cross entropy -> backward into the
//     critic and the encoder -> Adam on (encoder, critic) fused with target EMA
//   temperature step on log alpha
//   [actor step] updated critic scores the sampled action -> expected-Q gradient
//     -> backward to the action only -> policy backward -> Adam on the actor
//   statistics row, counters
// Everything that changes between updates (update index, Adam step counts)
// lives in device counters, so a captured graph is replayed unchanged.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ops.h"
#include "kernels/sample.h"
#include "kernels/finish.h"

namespace sq {

void plan_act(const Net& net, int n, Bump& b, ActBufs* w) {
  w->x = b.take<float>((size_t)n * net.img);
  plan_encoder(net, n, b, &w->e, false);
  plan_actor(net, n, b, &w->a, false);
  w->noise = b.take<float>((size_t)n * net.d.action);
}

int enqueue_act(const Net& net, const Layout& L, const sq_hparams& hp, const float* params, const float* pack,
                const ActBufs& w, const uint8_t* frames, const float* proprio, int n, int sample,
                unsigned long long request_id, float* action_out, hipStream_t st) {
  const sq_dims& d = net.d;
  const int bf = hp.prec == SQ_BF16;
  const float* feat = proprio;   // state-based: the state is the feature
  if (d.n_conv > 0) {
    SQ_TRY(launch_squint(frames, nullptr, n, d.H, d.W, d.C, d.k, 0, w.x, net.img, st));
    SQ_TRY(encoder_forward(net, bf, params, L, w.x, n, w.e, st));
    feat = w.e.h[d.n_conv - 1];
  }
  if (sample) SQ_TRY(launch_act_noise(hp.seed, request_id, n, d.action, w.noise, st));
  return actor_forward(net, bf, params + L.actor_begin, pack, L, feat, net.flat, proprio, d.proprio,
                       sample ? w.noise : nullptr, n, hp.log_std_min, hp.log_std_max, action_out, nullptr, w.a, st);
}

size_t act_bytes_per_obs(const Net& net) {
  Bump b{nullptr};
  ActBufs w;
  plan_act(net, 1024, b, &w);
  return (b.off + 1023) / 1024;
}

}  // namespace sq

using namespace sq;

// A captured block of updates.  The graph writes its statistics rows into a
// buffer of its own and copies them out in its last node, whose destination is
// set to the caller's pointer before a launch (only when it changed), so the
// caller's stats pointer is not part of the key.
struct GraphEntry {
  int n_updates, phase;
  sq_replay rep;          // compared field by field (the struct has padding)
  hipStream_t stream;
  hipGraph_t graph;       // kept for the copy node's handle
  hipGraphExec_t exec;
  hipGraphNode_t copy_node;
  hipKernelNodeParams copy_params;
  float* stats;           // [n_updates, 8], library-owned
  float* dst;             // destination of the copy node at the last launch
  unsigned long long last_use;
};

static void destroy_entry(GraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  if (e.stats) (void)hipFree(e.stats);
}
constexpr size_t kMaxGraphs = 8;   // least recently used graph evicted beyond this

static bool same_replay(const sq_replay& a, const sq_replay& b) {
  return a.obs == b.obs && a.next_obs == b.next_obs && a.proprio == b.proprio && a.next_proprio == b.next_proprio &&
         a.action == b.action && a.reward == b.reward && a.done == b.done && a.capacity == b.capacity &&
         a.size == b.size && a.squinted == b.squinted && a.dev_size == b.dev_size;
}

struct sq_agent {
  Net net;
  Layout L;
  sq_hparams hp;
  int B;
  float *params, *target, *m, *v, *grads;
  float *pack, *tpack;   // packed linear weights of params and of the target critic
  int* ctr;
  void* ws = nullptr;
  void* wsh = nullptr;   // bfloat16 copies of the products' operands (bfloat16 mode)
  bool own_grads = false;
  long long u_host = 0;
  // update buffers
  int* idx;
  float *eps2B, *S2, *r, *dn, *x, *dfeat, *act2B, *logp2B, *logits_t, *logits, *logits_q, *mt, *dlogits,
      *dlogits_q, *loss_row, *q_row, *tgt_row, *qa_row, *scal, *da;
  int* ta_snap;   // the actor Adam's step count, recorded by the critic Adam launch
  int dlp;        // row stride of dlogits / dlogits_q (the atoms rounded up to 8: 16-byte aligned rows)
  EncBufs enc;
  ActorBufs actor;
  CriticBufs crit, aux;
  // act()
  int act_cap;
  ActBufs actw;
  std::vector<GraphEntry> graphs;
  unsigned long long graph_clock = 0;
  long long graphs_captured = 0;
  PackArgs pk_critic, pk_actor;   // pack refresh tables of the two Adam launches
  GradSegs gs_critic, gs_actor;   // bias / gain / shift gradients the Adam launches sum from partials
  bool enc_seg = false;           // gs_critic also sums the fused encoder's partial gradients
  EncPrepMap enc_map{};           // the critic Adam keeps enc.wprep current (enc_map.n > 0)
};

static size_t plan_agent(sq_agent* g, char* base) {
  const Net& net = g->net;
  const sq_dims& d = net.d;
  const int B = g->B, A = d.action, S = d.proprio, N = d.atoms;
  Bump b{base};
  g->idx = b.take<int>(B);
  g->eps2B = b.take<float>((size_t)2 * B * A);
  g->S2 = b.take<float>((size_t)2 * B * (S > 0 ? S : 1));
  g->r = b.take<float>(B);
  g->dn = b.take<float>(B);
  g->x = b.take<float>((size_t)2 * B * net.img);
  plan_encoder(net, 2 * B, b, &g->enc, true);
  g->dfeat = b.take<float>((size_t)B * net.flat);
  g->act2B = b.take<float>((size_t)2 * B * A);
  g->logp2B = b.take<float>((size_t)2 * B);
  plan_actor(net, 2 * B, b, &g->actor, true);
  plan_critic(net, B, b, &g->crit, true, 2);
  plan_critic(net, B, b, &g->aux, true);
  g->logits = b.take<float>((size_t)4 * B * N);     // online twins, then target twins
  g->logits_t = g->logits ? g->logits + (size_t)2 * B * N : nullptr;
  g->logits_q = b.take<float>((size_t)2 * B * N);
  g->mt = b.take<float>((size_t)B * N);
  g->dlp = N > 1 ? (N + 7) / 8 * 8 : N;
  g->dlogits = b.take<float>((size_t)2 * B * g->dlp);
  g->dlogits_q = b.take<float>((size_t)2 * B * g->dlp);
  g->loss_row = b.take<float>((size_t)2 * B);
  g->q_row = b.take<float>((size_t)2 * B);
  g->tgt_row = b.take<float>(B);
  g->qa_row = b.take<float>(B);
  g->scal = b.take<float>(8);
  g->ta_snap = b.take<int>(1);
  g->da = b.take<float>((size_t)B * A);
  g->pack = b.take<float>(g->L.pack_total);
  g->tpack = b.take<float>(g->L.pack_critic_end);
  if (!g->own_grads) {
  } else {
    g->grads = b.take<float>(g->L.total);
  }
  plan_act(net, g->act_cap, b, &g->actw);
  return b.off + 256;
}

// In the bfloat16 mode the packed weights, every activation buffer that a product
// reads and the LayerNorm input gradients (dB) the backward products read get
// bfloat16 copies, kept by their producers (LayerNorm forward and backward, the
// fused encoder, the minibatch draw, the policy head, pack and Adam), so those
// products read half the bytes; so do the heads' gradients (dlogits, dhead, rows
// padded to 16-byte multiples), written by the cross-entropy, expected-Q and
// policy-head backward kernels.  Only buffers whose every producer writes the copy
// are registered (the products' own outputs, dA and dX1, are read by LayerNorm
// only and have none).
static int make_twins(sq_agent* g) {
  const Net& net = g->net;
  const sq_dims& d = net.d;
  const size_t B = (size_t)g->B, H = (size_t)d.hidden, w = (size_t)std::max(d.hidden, d.proj);
  struct Item { const float* f; size_t n; };
  std::vector<Item> items = {
      {g->pack, (size_t)g->L.pack_total}, {g->tpack, (size_t)g->L.pack_critic_end},
      {g->crit.X1, 2 * B * net.cpad},     {g->crit.g1, 4 * B * H},  {g->crit.g2, 4 * B * H},
      {g->aux.X1, B * net.cpad},          {g->aux.g1, 2 * B * H},   {g->aux.g2, 2 * B * H},
      {g->actor.X1, 2 * B * net.apad},    {g->actor.g1, 2 * B * H}, {g->actor.g2, 2 * B * H},
      {g->crit.dB, 2 * B * w},            {g->aux.dB, 2 * B * w},   {g->actor.dB, 2 * B * w},
      {g->actor.dhead, 2 * B * (size_t)g->actor.ldh}};
  if (d.atoms > 1) {   // the C51 heads' gradients (the scalar heads' have one column)
    items.push_back({g->dlogits, 2 * B * (size_t)g->dlp});
    items.push_back({g->dlogits_q, 2 * B * (size_t)g->dlp});
  }
  if (d.n_conv > 0 && encoder_fused(net, 1, g->enc)) items.push_back({g->enc.h[d.n_conv - 1], 2 * B * net.flat});
  Bump b{nullptr};
  for (const Item& it : items) b.take<uint16_t>(it.n);
  const size_t bytes = b.off + 256;
  if (hipMalloc(&g->wsh, bytes) != hipSuccess) {
    g->wsh = nullptr;
    set_error("hipMalloc of %zu bytes for the bfloat16 operand copies failed", bytes);
    return SQ_ENOMEM;
  }
  SQ_TRY_HIP(hipMemset(g->wsh, 0, bytes));
  Bump h{(char*)(((uintptr_t)g->wsh + 255) & ~(uintptr_t)255)};
  for (const Item& it : items) twin_register(g, it.f, (long long)it.n, h.take<uint16_t>(it.n));
  // the hidden layers' ReLU outputs are read through their copies only (the
  // products read the copies; the LayerNorm backward recomputes the ReLU mask), so
  // their FP32 values are not kept.  That needs rows the copy loads can read (a
  // width that is a multiple of 8) and, for the critics' second layer, a copy of
  // the head gradient its weight gradient is taken against (the C51 heads)
  if (H % 8 == 0) {
    std::vector<Item> drop = {{g->crit.g1, 4 * B * H}, {g->aux.g1, 2 * B * H},  {g->aux.g2, 2 * B * H},
                              {g->actor.g1, 2 * B * H}, {g->actor.g2, 2 * B * H}};
    if (d.atoms > 1) drop.push_back({g->crit.g2, 4 * B * H});
    for (const Item& it : drop) fp32_drop_register(g, it.f, (long long)it.n);
  }
  // the target critic's packed weights are read only by the target batches of the
  // critic products, through their copies, where the inputs are images (the
  // state-based first layer reads the sampled states, which have no copy)
  if (H % 8 == 0 && d.n_conv > 0) {
    fp32_drop_register(g, g->tpack, (long long)g->L.pack_critic_end);
    g->pk_critic.tpack32 = 0;
  }
  g->pk_critic.pack_h = g->pk_actor.pack_h = twin_of(g->pack, g->L.pack_total);
  g->pk_critic.tpack_h = twin_of(g->tpack, g->L.pack_critic_end);
  return SQ_OK;
}

static void free_agent(sq_agent* g) {
  twin_unregister(g);
  if (g->wsh) (void)hipFree(g->wsh);
  if (g->ws) (void)hipFree(g->ws);
  delete g;
}

static int enqueue_update(sq_agent* g, const sq_replay* R, float* stats, int actor_step, hipStream_t st) {
  const Net& net = g->net;
  const sq_dims& d = net.d;
  const Layout& L = g->L;
  const sq_hparams& hp = g->hp;
  const int B = g->B, A = d.action, S = d.proprio, N = d.atoms, flat = net.flat;
  const int bf = hp.prec == SQ_BF16;
  const float lo = hp.log_std_min, hi = hp.log_std_max;
  float* P = g->params;
  float* G = g->grads;
  // the critics' input rows [projection | s | a] (batch 0: online on s, batch 1:
  // target on s'): the replayed actions go straight into batch 0's action columns,
  // the target policy's actions into batch 1's (written by the policy head)
  const int cld = net.cpad;
  float* xa_online = g->crit.X1 + d.proj + S;
  float* xa_target = g->crit.X1 + (size_t)B * cld + d.proj + S;
  const SampleArgs sa = sample_args(hp.seed, g->ctr, R->size, R->dev_size, B, A, S, R->proprio, R->next_proprio,
                                    R->action, R->reward, R->done, g->idx, g->eps2B, g->S2, xa_online, cld, g->r,
                                    g->dn);
  // state-based SAC: the sampled states [s; s'] (S2) are the features
  const bool image = d.n_conv > 0;
  const float* feat = g->S2;
  // in bfloat16 the draw and the squint run inside the encoder's launch where the geometry allows
  int fused = kNotApplicable;
  if (image && bf)
    fused = encoder_forward_squint(net, P, L, sa, R->obs, R->next_obs, g->x, g->enc, st, g->enc_map.n > 0,
                                   R->squinted != 0);
  if (fused != kNotApplicable) SQ_TRY(fused);
  if (fused == kNotApplicable && (!image || R->squinted)) SQ_TRY(launch_sample_batch(sa, st));
  if (image && fused == kNotApplicable) {
    // frames squinted at insertion are the k = 1 squint of the stored block means;
    // raw frames are drawn and squinted in one launch
    if (R->squinted)
      SQ_TRY(launch_squint_pair(R->obs, R->next_obs, g->idx, B, net.side, net.side, d.C, 1, g->x, st));
    else
      SQ_TRY(launch_sample_squint(sa, R->obs, R->next_obs, d.H, d.W, d.C, d.k, g->x, st));
    SQ_TRY(encoder_forward(net, bf, P, L, g->x, 2 * B, g->enc, st, g->enc_map.n > 0));
  }
  if (image) feat = g->enc.h[d.n_conv - 1];
  SQ_TRY(trunks_forward(net, bf, P + L.actor_begin, P + L.critic_begin, g->target, g->pack, g->pack, g->tpack, L,
                        feat, flat, g->S2, S, B, g->actor, g->crit, st));
  ActorBufs ab = g->actor;
  ab.xact = xa_target;
  ab.ld_xact = cld;
  ab.xact_row0 = B;
  SQ_TRY(actor_forward(net, bf, P + L.actor_begin, g->pack, L, feat, flat, g->S2, S, g->eps2B, 2 * B, lo, hi,
                       g->act2B, g->logp2B, ab, st, true));
  // online critics on (z, s, a) and target critics on (z', s', a~') in one pass;
  // their input rows are complete (projections, states and both action blocks)
  SQ_TRY(critic_forward_pair(net, bf, P + L.critic_begin, g->target, g->pack, g->tpack, L, feat, flat,
                             (long long)B * flat, g->S2, S, (long long)B * S, nullptr, nullptr, A, B, g->logits,
                             g->crit, st, true));
  // distributional soft target from the averaged twin target critics (projection),
  // and the online critics' cross entropy to it, in one pass over the rows
  if (N == 1)
    SQ_TRY(target_mse(g->logits, B, g->r, g->dn, g->logp2B + B, P + L.log_alpha, hp.gamma, hp.cdq, g->tgt_row,
                      g->dlogits, g->loss_row, g->q_row, g->crit.part_out, st));
  else
    SQ_TRY(target_ce(g->logits, B, N, d.v_min, d.v_max, g->r, g->dn, g->logp2B + B, P + L.log_alpha, hp.gamma,
                     hp.cdq, g->mt, g->tgt_row, g->dlogits, g->loss_row, g->q_row, g->crit.part_out, st, g->dlp));
  SQ_TRY(critic_backward(net, bf, P + L.critic_begin, g->pack, L, feat, flat, g->dlogits, B, g->crit, G + L.critic_begin,
                         image ? g->dfeat : nullptr, nullptr, st, true, true, nullptr, g->dlp));
  // the fused encoder's partial gradients are summed by the critic Adam launch
  if (image) SQ_TRY(encoder_backward(net, bf, P, L, g->x, B, g->dfeat, g->enc, G, st, true, g->enc_seg));
  // critic + encoder Adam (with the target EMA and the packed copies), and the
  // temperature step in one extra workgroup of the same launch
  const AlphaJob aj{g->logp2B, B, hp.target_entropy, P + L.log_alpha, G + L.log_alpha, g->m + L.log_alpha,
                    g->v + L.log_alpha, g->ctr, g->scal, actor_step ? g->ta_snap : nullptr};
  SQ_TRY(adam(P, G, g->m, g->v, L.critic_end, &hp, g->ctr + CTR_TC, g->target, L.critic_begin, nullptr, &g->pk_critic,
              st, &g->gs_critic, &aj, g->enc_map.n > 0 ? &g->enc_map : nullptr));
  // delayed actor step against the updated critic
  if (actor_step) {
    SQ_TRY(critic_forward(net, bf, P + L.critic_begin, g->pack, L, feat, flat, g->S2, S, g->act2B, A, B, g->logits_q,
                          g->aux, st));
    if (N == 1)
      SQ_TRY(expected_q_scalar(g->logits_q, B, g->dlogits_q, g->qa_row, st));
    else
      SQ_TRY(expected_q_grad(g->logits_q, B, N, d.v_min, d.v_max, g->dlogits_q, g->qa_row, st, g->dlp));
    // the policy head's backward (d log pi scaled by the updated alpha / B) runs as
    // the epilogue of the critic product that forms dQ/da
    const TgBwdJob tj{g->actor.save, g->eps2B, nullptr, g->scal + 1, 1.0f / (float)B, lo, hi, g->actor.dhead,
                      g->actor.part_out, g->actor.ldh};
    SQ_TRY(critic_backward(net, bf, P + L.critic_begin, g->pack, L, feat, flat, g->dlogits_q, B, g->aux, nullptr, nullptr,
                           g->da, st, false, false, &tj, g->dlp));
    SQ_TRY(actor_backward(net, bf, P + L.actor_begin, g->pack, L, feat, flat, g->eps2B, B, g->da, A, nullptr, g->scal + 1,
                          1.0f / (float)B, lo, hi, g->actor, G + L.actor_begin, st, true, true));
    // the actor Adam launch also ends the update in its first workgroup; its step
    // count is the one the critic launch recorded, since that workgroup advances
    // the counters
    const FinishJob fj{g->loss_row, g->q_row, g->tgt_row, g->logp2B, g->qa_row, g->scal, B, 1, g->ctr, stats};
    return adam(P + L.actor_begin, G + L.actor_begin, g->m + L.actor_begin, g->v + L.actor_begin,
                L.actor_end - L.actor_begin, &hp, g->ta_snap, nullptr, 0, nullptr, &g->pk_actor, st, &g->gs_actor,
                nullptr, nullptr, &fj);
  }
  return finish_update(g->loss_row, g->q_row, g->tgt_row, g->logp2B, g->qa_row, g->scal, B, 0, g->ctr, stats, st);
}

static int check_replay(const sq_agent* g, const sq_replay* R) {
  if (!R) { set_error("replay is NULL"); return SQ_EINVAL; }
  if ((g->net.d.n_conv > 0 && (!R->obs || !R->next_obs)) || !R->action || !R->reward || !R->done ||
      (g->net.d.proprio > 0 && (!R->proprio || !R->next_proprio))) {
    set_error("replay has a NULL field");
    return SQ_EINVAL;
  }
  if (R->size <= 0 || R->size > R->capacity) {
    set_error("replay size %d outside (0, capacity=%d]", R->size, R->capacity);
    return SQ_EINVAL;
  }
  if (R->squinted != 0 && R->squinted != 1) {
    set_error("replay squinted flag %d is neither 0 nor 1", R->squinted);
    return SQ_EINVAL;
  }
  return SQ_OK;
}

static int enqueue_block(sq_agent* g, const sq_replay* R, int n, float* stats, hipStream_t st) {
  const int pf = g->hp.policy_freq;
  for (int j = 0; j < n; ++j) {
    const int actor_step = ((g->u_host + j) % pf) == 0;
    SQ_TRY(enqueue_update(g, R, stats + 8 * (size_t)j, actor_step, st));
  }
  return SQ_OK;
}

extern "C" {

int sq_agent_create(const sq_dims* dims, const sq_hparams* hp, int batch, float* params, float* target,
                    float* adam_m, float* adam_v, float* grads, int* counters, sq_agent** out) {
  Net net;
  SQ_TRY(make_net(dims, &net));
  if (!hp || !out || !params || !target || !adam_m || !adam_v || !counters) {
    set_error("NULL argument to sq_agent_create");
    return SQ_EINVAL;
  }
  if (batch <= 0 || hp->policy_freq <= 0 || (hp->prec != SQ_F32 && hp->prec != SQ_BF16)) {
    set_error("bad batch %d / policy_freq %d / prec", batch, hp->policy_freq);
    return SQ_EINVAL;
  }
  if (hp->cdq != 0 && hp->cdq != 1) {
    set_error("cdq %d is neither 0 nor 1", hp->cdq);
    return SQ_EINVAL;
  }
  if (!(hp->gamma >= 0.f && hp->gamma <= 1.f)) {
    set_error("discount gamma %g outside [0, 1]", (double)hp->gamma);
    return SQ_EINVAL;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
    set_error("sq_agent_create allocates and cannot run while the null stream captures");
    return SQ_ECAPTURE;
  }
  sq_agent* g = new sq_agent();
  g->net = net;
  make_layout(net, &g->L);
  g->hp = *hp;
  g->B = batch;
  g->params = params;
  g->target = target;
  g->m = adam_m;
  g->v = adam_v;
  g->grads = grads;
  g->own_grads = grads == nullptr;
  g->ctr = counters;
  g->act_cap = 4096;
  const size_t bytes = plan_agent(g, nullptr);
  if (hipMalloc(&g->ws, bytes) != hipSuccess) {
    delete g;
    set_error("hipMalloc of %zu workspace bytes failed", bytes);
    return SQ_ENOMEM;
  }
  char* base = (char*)(((uintptr_t)g->ws + 255) & ~(uintptr_t)255);
  plan_agent(g, base);
  {
    const Layout& L = g->L;
    g->pk_critic = PackArgs{};
    g->pk_actor = PackArgs{};
    for (int i = 0; i < L.n_pack; ++i) {
      PackArgs& t = L.pack[i].critic ? g->pk_critic : g->pk_actor;
      t.seg[t.n++] = L.pack[i];
    }
    g->pk_critic.pack = g->pk_actor.pack = g->pack;
    g->pk_critic.tpack = g->tpack;
    g->pk_critic.p_begin = 0;
    g->pk_actor.p_begin = L.actor_begin;
    critic_grad_segs(g->net, L, g->crit, g->B, &g->gs_critic);
    if (g->net.d.n_conv > 0)
      (void)encoder_fused_prep_map(g->net.d.C, g->net.d.F, g->net.d.n_conv, g->net.side, L.conv_W, g->enc.wprep,
                                   hp->prec == SQ_BF16, &g->enc_map);
    GradSeg es;
    if (encoder_grad_seg(g->net, hp->prec == SQ_BF16, L, g->enc, g->B, &es)) {
      // the encoder block comes first in the flat vector, so the list stays sorted
      for (int i = g->gs_critic.n; i > 0; --i) g->gs_critic.s[i] = g->gs_critic.s[i - 1];
      g->gs_critic.s[0] = es;
      ++g->gs_critic.n;
      g->enc_seg = true;
    }
    actor_grad_segs(g->net, L, g->actor, g->B, &g->gs_actor);
    g->gs_critic.gout = g->grads;
    g->gs_actor.gout = g->grads + L.actor_begin;
  }
  if (hp->prec == SQ_BF16 && twins_enabled()) {
    const int s = make_twins(g);
    if (s != SQ_OK) {
      free_agent(g);
      return s;
    }
  }
  if (pack_weights(g->L, params, target, g->pack, g->tpack, nullptr) != SQ_OK ||
      encoder_prepare(g->net, hp->prec == SQ_BF16, params, g->L, g->enc, nullptr) != SQ_OK ||
      hipDeviceSynchronize() != hipSuccess) {
    free_agent(g);
    return SQ_EDEVICE;
  }
  int host_ctr[CTR_N];
  if (hipMemcpy(host_ctr, counters, sizeof(host_ctr), hipMemcpyDeviceToHost) != hipSuccess) {
    free_agent(g);
    set_error("reading the counters failed");
    return SQ_EDEVICE;
  }
  g->u_host = host_ctr[CTR_U];
  *out = g;
  return SQ_OK;
}

int sq_agent_destroy(sq_agent* g) {
  if (!g) return SQ_OK;
  if (!g->graphs.empty()) (void)hipDeviceSynchronize();
  for (auto& e : g->graphs) destroy_entry(e);
  free_agent(g);
  return SQ_OK;
}

int sac_update_eager(sq_agent* g, const sq_replay* R, int n_updates, float* stats, sq_stream_t stream) {
  if (!g || !stats || n_updates < 0) {
    set_error("bad agent / stats / n_updates");
    return SQ_EINVAL;
  }
  SQ_TRY(check_replay(g, R));
  SQ_TRY(enqueue_block(g, R, n_updates, stats, (hipStream_t)stream));
  g->u_host += n_updates;
  return SQ_OK;
}

// Capture n updates and the statistics copy on st into e (graph, exec, copy node).
static int capture_block(sq_agent* g, const sq_replay* R, int n, hipStream_t st, GraphEntry* e) {
  hipError_t he = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) {
    set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(he));
    return SQ_EDEVICE;
  }
  int s = enqueue_block(g, R, n, e->stats, st);
  if (s == SQ_OK) s = launch_copy_stats(e->stats, e->dst, 8 * n, st);
  const hipError_t ce = hipStreamEndCapture(st, &e->graph);
  if (s != SQ_OK) return s;
  if (ce != hipSuccess) {
    set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ce));
    return SQ_EDEVICE;
  }
  // find the copy node (the only launch of its kernel in the graph)
  size_t nn = 0;
  SQ_TRY_HIP(hipGraphGetNodes(e->graph, nullptr, &nn));
  std::vector<hipGraphNode_t> nodes(nn);
  SQ_TRY_HIP(hipGraphGetNodes(e->graph, nodes.data(), &nn));
  e->copy_node = nullptr;
  for (size_t i = 0; i < nn; ++i) {
    hipGraphNodeType t;
    SQ_TRY_HIP(hipGraphNodeGetType(nodes[i], &t));
    if (t != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    SQ_TRY_HIP(hipGraphKernelNodeGetParams(nodes[i], &kp));
    if (kp.func == copy_stats_kernel()) {
      e->copy_node = nodes[i];
      e->copy_params = kp;
    }
  }
  if (!e->copy_node) {
    set_error("the captured graph has no statistics copy node");
    return SQ_EDEVICE;
  }
  const hipError_t ie = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    e->exec = nullptr;
    set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
    return SQ_EDEVICE;
  }
  return SQ_OK;
}

int sac_update(sq_agent* g, const sq_replay* R, int n_updates, float* stats, sq_stream_t stream) {
  if (!g || !stats || n_updates < 0) {
    set_error("bad agent / stats / n_updates");
    return SQ_EINVAL;
  }
  SQ_TRY(check_replay(g, R));
  if (n_updates == 0) return SQ_OK;
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  SQ_TRY_HIP(hipStreamIsCapturing(st, &cs));
  if (st == nullptr || cs != hipStreamCaptureStatusNone) {
    // the null stream cannot be captured; inside a caller's capture the
    // kernels simply become part of the caller's graph
    return sac_update_eager(g, R, n_updates, stats, stream);
  }
  const int phase = (int)(g->u_host % g->hp.policy_freq);
  GraphEntry* hit = nullptr;
  for (auto& e : g->graphs)
    if (e.n_updates == n_updates && e.phase == phase && e.stream == st && same_replay(e.rep, *R)) hit = &e;
  if (!hit) {
    if (g->graphs.size() >= kMaxGraphs) {
      // evict the least recently used graph; its launches may still be in flight
      size_t old = 0;
      for (size_t i = 1; i < g->graphs.size(); ++i)
        if (g->graphs[i].last_use < g->graphs[old].last_use) old = i;
      SQ_TRY_HIP(hipDeviceSynchronize());
      destroy_entry(g->graphs[old]);
      g->graphs.erase(g->graphs.begin() + (long)old);
    }
    GraphEntry e{};
    e.n_updates = n_updates;
    e.phase = phase;
    e.rep = *R;
    e.stream = st;
    e.dst = stats;
    if (hipMalloc(&e.stats, sizeof(float) * 8 * (size_t)n_updates) != hipSuccess) {
      set_error("hipMalloc of the graph's %d statistics rows failed", n_updates);
      return SQ_ENOMEM;
    }
    const int s = capture_block(g, R, n_updates, st, &e);
    if (s != SQ_OK) {
      destroy_entry(e);
      return s;
    }
    g->graphs.push_back(e);
    ++g->graphs_captured;
    hit = &g->graphs.back();
  }
  hit->last_use = ++g->graph_clock;
  if (hit->dst != stats) {
    // point the copy node at this call's stats buffer
    const float* src = hit->stats;
    float* dst = stats;
    int n = 8 * n_updates;
    void* args[] = {&src, &dst, &n};
    hipKernelNodeParams kp = hit->copy_params;
    kp.kernelParams = args;
    SQ_TRY_HIP(hipGraphExecKernelNodeSetParams(hit->exec, hit->copy_node, &kp));
    hit->dst = stats;
  }
  SQ_TRY_HIP(hipGraphLaunch(hit->exec, st));
  g->u_host += n_updates;
  return SQ_OK;
}

int sq_agent_graph_count(const sq_agent* g, long long* captured, int* cached) {
  if (!g || !captured || !cached) { set_error("NULL argument to sq_agent_graph_count"); return SQ_EINVAL; }
  *captured = g->graphs_captured;
  *cached = (int)g->graphs.size();
  return SQ_OK;
}

int sq_agent_last_indices(const sq_agent* g, int* idx, sq_stream_t stream) {
  if (!g || !idx) { set_error("NULL argument to sq_agent_last_indices"); return SQ_EINVAL; }
  SQ_TRY_HIP(hipMemcpyAsync(idx, g->idx, sizeof(int) * (size_t)g->B, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SQ_OK;
}

int sq_agent_last_target(const sq_agent* g, float* m, sq_stream_t stream) {
  if (!g || !m) { set_error("NULL argument to sq_agent_last_target"); return SQ_EINVAL; }
  if (g->net.d.atoms < 2) {
    set_error("sq_agent_last_target: scalar critics have no target distribution");
    return SQ_EINVAL;
  }
  SQ_TRY_HIP(hipMemcpyAsync(m, g->mt, sizeof(float) * (size_t)g->B * g->net.d.atoms, hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
  return SQ_OK;
}

int act(sq_agent* g, const uint8_t* frames, const float* proprio, int n, int sample, unsigned long long request_id,
        float* action_out, sq_stream_t stream) {
  if (!g) { set_error("agent is NULL"); return SQ_EINVAL; }
  if (n < 0 || n > g->act_cap) {
    set_error("n = %d outside [0, %d]", n, g->act_cap);
    return SQ_EINVAL;
  }
  if (n == 0) return SQ_OK;
  if ((g->net.d.n_conv > 0 && !frames) || !action_out || (g->net.d.proprio > 0 && !proprio)) {
    set_error("NULL argument to act");
    return SQ_EINVAL;
  }
  return enqueue_act(g->net, g->L, g->hp, g->params, g->pack, g->actw, frames, proprio, n, sample ? 1 : 0,
                     request_id, action_out, (hipStream_t)stream);
}

int sq_agent_sync(sq_agent* g, sq_stream_t stream) {
  if (!g) { set_error("agent is NULL"); return SQ_EINVAL; }
  SQ_TRY(pack_weights(g->L, g->params, g->target, g->pack, g->tpack, (hipStream_t)stream));
  return encoder_prepare(g->net, g->hp.prec == SQ_BF16, g->params, g->L, g->enc, (hipStream_t)stream);
}

int sq_agent_act_capacity(sq_agent* g, int* n) {
  if (!g || !n) { set_error("NULL argument"); return SQ_EINVAL; }
  *n = g->act_cap;
  return SQ_OK;
}

}  // extern "C"

// used by the serving loop
namespace sq {
const Net& agent_net(const sq_agent* g) { return g->net; }
const Layout& agent_layout(const sq_agent* g) { return g->L; }
const sq_hparams& agent_hp(const sq_agent* g) { return g->hp; }
const float* agent_params(const sq_agent* g) { return g->params; }
const float* agent_pack(const sq_agent* g) { return g->pack; }
}  // namespace sq
