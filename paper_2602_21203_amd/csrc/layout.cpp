// Dimension checks and the canonical flat parameter layout.
//
// Order: encoder convs {W[F, Cin, 3, 3], b} (none in the state-based form, whose
// features are the proprio state); critic projection {W[proj, flat],
// b, ln gain, ln shift}; twin critics q1, q2 each {l1 W[hidden, proj+P+A], b,
// gain, shift; l2 W[hidden, hidden], b, gain, shift; out W[atoms, hidden], b};
// actor projection (critic projection shapes); actor {l1 W[hidden, proj+P], ...,
// out W[2A, hidden], b}; log alpha.
#include <stdarg.h>
#include <stdio.h>

#include "common.h"

namespace sq {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char* last_error() { return g_err; }

int make_net(const sq_dims* d, Net* n) {
  if (!d) { set_error("dims is NULL"); return SQ_EINVAL; }
  if (d->n_conv == 0) {
    // state-based SAC (no image, no encoder): the proprio vector is the state
    // and takes the place of the encoder features; the frame fields are unused
    if (d->proprio <= 0 || d->proj <= 0 || d->hidden <= 0 || d->action <= 0 || d->atoms < 1) {
      set_error("bad state-based dims proprio=%d proj=%d hidden=%d atoms=%d action=%d", d->proprio, d->proj,
                d->hidden, d->atoms, d->action);
      return SQ_EINVAL;
    }
    if (d->proj > 1024 || d->hidden > 1024 || d->atoms > 256) {
      set_error("widths above the kernel limits (proj, hidden <= 1024, atoms <= 256)");
      return SQ_EINVAL;
    }
    if (d->atoms > 1 && !(d->v_max > d->v_min)) { set_error("need v_max > v_min"); return SQ_EINVAL; }
    *n = Net{};
    n->d = *d;
    n->flat = d->proprio;
    n->cin_critic = d->proj + d->proprio + d->action;
    n->cin_actor = d->proj + d->proprio;
    n->cpad = (n->cin_critic + 7) / 8 * 8;
    n->apad = (n->cin_actor + 7) / 8 * 8;
    return SQ_OK;
  }
  if (d->C <= 0 || d->H <= 0 || d->W <= 0 || d->k <= 0 || d->H % d->k || d->W % d->k || d->H != d->W) {
    set_error("bad frame dims C=%d H=%d W=%d k=%d (need square frames with H %% k == 0)", d->C, d->H, d->W, d->k);
    return SQ_EINVAL;
  }
  if (d->n_conv < 1 || d->n_conv > 4 || d->F <= 0 || d->proj <= 0 || d->hidden <= 0 || d->proprio < 0 ||
      d->action <= 0 || d->atoms < 1) {
    set_error("bad network dims n_conv=%d F=%d proj=%d hidden=%d atoms=%d proprio=%d action=%d", d->n_conv, d->F,
              d->proj, d->hidden, d->atoms, d->proprio, d->action);
    return SQ_EINVAL;
  }
  if (d->proj > 1024 || d->hidden > 1024 || d->atoms > 256) {
    set_error("widths above the kernel limits (proj, hidden <= 1024, atoms <= 256)");
    return SQ_EINVAL;
  }
  if (d->atoms > 1 && !(d->v_max > d->v_min)) { set_error("need v_max > v_min"); return SQ_EINVAL; }
  if (!squint_ok(d->H, d->W, d->C, d->k)) {
    set_error("frame geometry %dx%dx%d / k=%d exceeds the squint kernel's tile", d->H, d->W, d->C, d->k);
    return SQ_EINVAL;
  }
  n->d = *d;
  n->side = d->H / d->k;
  int s = (n->side - 3) / 2 + 1;
  if (n->side < 3 || s < 1) { set_error("squinted side %d too small", n->side); return SQ_EINVAL; }
  n->conv_side[0] = s;
  for (int i = 1; i < d->n_conv; ++i) {
    s -= 2;
    if (s < 1) { set_error("conv stack too deep for a %d x %d input", n->side, n->side); return SQ_EINVAL; }
    n->conv_side[i] = s;
  }
  n->flat = d->F * s * s;
  n->cin_critic = d->proj + d->proprio + d->action;
  n->cin_actor = d->proj + d->proprio;
  n->cpad = (n->cin_critic + 7) / 8 * 8;
  n->apad = (n->cin_actor + 7) / 8 * 8;
  n->img = d->C * n->side * n->side;
  return SQ_OK;
}

void make_layout(const Net& n, Layout* L) {
  const sq_dims& d = n.d;
  long long off = 0;
  int t = 0;
  auto take = [&](long long count) {
    L->tensor_off[t++] = off;
    const long long o = off;
    off += count;
    return o;
  };
  L->enc_begin = 0;
  int cin = d.C;
  for (int i = 0; i < d.n_conv; ++i) {
    L->conv_W[i] = take((long long)d.F * cin * 9);
    L->conv_b[i] = take(d.F);
    cin = d.F;
  }
  L->enc_end = L->critic_begin = off;
  auto dense = [&](int out, int in) {
    Dense x;
    x.out = out;
    x.in = in;
    x.W = take((long long)out * in);
    x.b = take(out);
    x.g = take(out);
    x.beta = take(out);
    return x;
  };
  auto head = [&](int out, int in) {
    Head x;
    x.out = out;
    x.in = in;
    x.W = take((long long)out * in);
    x.b = take(out);
    return x;
  };
  L->ctrunk = dense(d.proj, n.flat);
  for (int q = 0; q < 2; ++q) {
    L->q[q].l1 = dense(d.hidden, n.cin_critic);
    L->q[q].l2 = dense(d.hidden, d.hidden);
    L->q[q].out = head(d.atoms, d.hidden);
  }
  L->critic_end = L->actor_begin = off;
  L->atrunk = dense(d.proj, n.flat);
  L->al1 = dense(d.hidden, n.cin_actor);
  L->al2 = dense(d.hidden, d.hidden);
  L->aout = head(2 * d.action, d.hidden);
  L->actor_end = off;
  L->log_alpha = take(1);
  L->total = off;
  L->n_tensors = t;
  L->tensor_off[t] = off;
  // packed copy of the linear weights
  long long poff = 0;
  L->n_pack = 0;
  auto pk = [&](long long src, int rows, int cols, int critic, long long* Wp, int* ldp) {
    const int ld = (cols + 7) / 8 * 8;
    poff = (poff + 63) / 64 * 64;
    L->pack[L->n_pack++] = PackSeg{src, poff, rows, cols, ld, critic};
    *Wp = poff;
    *ldp = ld;
    poff += (long long)rows * ld;
  };
  pk(L->ctrunk.W, L->ctrunk.out, L->ctrunk.in, 1, &L->ctrunk.Wp, &L->ctrunk.ldp);
  for (int q = 0; q < 2; ++q) {
    Twin& tq = L->q[q];
    pk(tq.l1.W, tq.l1.out, tq.l1.in, 1, &tq.l1.Wp, &tq.l1.ldp);
    pk(tq.l2.W, tq.l2.out, tq.l2.in, 1, &tq.l2.Wp, &tq.l2.ldp);
    pk(tq.out.W, tq.out.out, tq.out.in, 1, &tq.out.Wp, &tq.out.ldp);
  }
  L->pack_critic_end = (poff + 63) / 64 * 64;
  pk(L->atrunk.W, L->atrunk.out, L->atrunk.in, 0, &L->atrunk.Wp, &L->atrunk.ldp);
  pk(L->al1.W, L->al1.out, L->al1.in, 0, &L->al1.Wp, &L->al1.ldp);
  pk(L->al2.W, L->al2.out, L->al2.in, 0, &L->al2.Wp, &L->al2.ldp);
  pk(L->aout.W, L->aout.out, L->aout.in, 0, &L->aout.Wp, &L->aout.ldp);
  L->pack_total = (poff + 63) / 64 * 64;
}

}  // namespace sq
