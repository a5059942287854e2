"""torch.autograd.Function wrappers over the library's hand-written backward.

EncoderFn, CriticFn and ActorFn make the encoder, the twin critics and the
tanh-Gaussian actor composable with torch autograd: forward calls the
library's *_fwd entry point and keeps its workspace; backward calls the
matching *_bwd entry point.  Every computation runs in libsquint's kernels.

Gradients flow to: the encoder parameters (not to the image); the critic
parameters, features and action; the actor parameters and, through the sampled
action and log-probability, nowhere else (features and noise are treated as
constants, as in the update where the actor sees stop-gradient features).
"""
import torch

from . import _lib as L
from . import api


class EncoderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, enc_params, x, cfg, prec):
        feat, ws = api.encoder_fwd(cfg, prec, enc_params, x.contiguous())
        ctx.save_for_backward(enc_params)
        ctx.ws, ctx.cfg, ctx.prec = ws, cfg, prec
        return feat

    @staticmethod
    def backward(ctx, dfeat):
        (enc_params,) = ctx.saved_tensors
        d = api.encoder_bwd(ctx.cfg, ctx.prec, enc_params, ctx.ws, dfeat.contiguous(), enc_params.numel())
        return d, None, None, None


class CriticFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, critic_params, feat, proprio, action, cfg, prec):
        logits, ws = api.critic_fwd(cfg, prec, critic_params, feat.contiguous(), proprio.contiguous(),
                                    action.contiguous())
        ctx.save_for_backward(critic_params)
        ctx.ws, ctx.cfg, ctx.prec = ws, cfg, prec
        return logits

    @staticmethod
    def backward(ctx, dlogits):
        (critic_params,) = ctx.saved_tensors
        need_p, need_f, _, need_a = ctx.needs_input_grad[:4]
        dp, df, da = api.critic_bwd(ctx.cfg, ctx.prec, critic_params, ctx.ws, dlogits.contiguous(),
                                    want_params=True, want_feat=need_f, want_action=need_a)
        return (dp if need_p else None), df, None, da, None, None


class ActorFn(torch.autograd.Function):
    """Returns (action, log_prob) of a reparameterised tanh-Gaussian sample."""

    @staticmethod
    def forward(ctx, actor_params, feat, proprio, eps, cfg, prec, hp):
        action, logp, ws = api.actor_fwd(cfg, prec, hp, actor_params, feat.contiguous(), proprio.contiguous(),
                                         eps.contiguous())
        ctx.save_for_backward(actor_params)
        ctx.ws, ctx.cfg, ctx.prec, ctx.hp = ws, cfg, prec, hp
        return action, logp

    @staticmethod
    def backward(ctx, daction, dlogp):
        (actor_params,) = ctx.saved_tensors
        # autograd materialises zero gradients for an unused output
        dp = api.actor_bwd(ctx.cfg, ctx.prec, ctx.hp, actor_params, ctx.ws, daction.contiguous(),
                           dlogp.contiguous())
        return dp, None, None, None, None, None, None


def encoder(enc_params, x, cfg, prec=L.SQ_F32):
    return EncoderFn.apply(enc_params, x, cfg, prec)


def critic(critic_params, feat, proprio, action, cfg, prec=L.SQ_F32):
    return CriticFn.apply(critic_params, feat, proprio, action, cfg, prec)


def actor(actor_params, feat, proprio, eps, cfg, hp, prec=L.SQ_F32):
    return ActorFn.apply(actor_params, feat, proprio, eps, cfg, prec, hp)
