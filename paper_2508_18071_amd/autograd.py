"""torch.autograd wrappers around the HIP forward/backward and the EMD loss.

``EvsFunction.apply(net, ckpt_every, x, *weights)`` runs the fused forward
(saving membrane checkpoints every ``ckpt_every`` frames) and returns the
spikes as float32; its backward calls the library's BPTT kernels.
``EmdLossFunction.apply(s, e, lambda_count)`` is the bidirectional EMD loss.
"""

from __future__ import annotations

import torch

from . import api


class EvsFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, net, ckpt_every, x, *weights):
        packed = api.pack_weights(net, [w.detach() for w in weights])
        out = api.forward(net, packed, x.detach(), s_fp32=True, ckpt_every=ckpt_every)
        ctx.net = net
        ctx.k = ckpt_every
        ctx.save_for_backward(x, out["ckpt"], packed)
        return out["s"]

    @staticmethod
    def backward(ctx, grad_s):
        x, ckpt, packed = ctx.saved_tensors
        want_dx = ctx.needs_input_grad[2]
        gws, dx, _ = api.backward(ctx.net, packed, x, ckpt, ctx.k, grad_s.contiguous(), want_dx=want_dx)
        return (None, None, dx, *gws)


class EmdLossFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, e, lambda_count=0.0):
        loss, g = api.emd_loss(s.detach().contiguous(), e, lambda_count, grad=True)
        ctx.save_for_backward(g)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_loss):
        (g,) = ctx.saved_tensors
        return g * grad_loss, None, None


def evsnet(net, x, weights, ckpt_every=16):
    """Differentiable EvSNet forward: spikes [N,T,Cout,H,W] float32."""
    return EvsFunction.apply(net, ckpt_every, x, *weights)


def emd_loss(s, e, lambda_count=0.0):
    return EmdLossFunction.apply(s, e, lambda_count)
