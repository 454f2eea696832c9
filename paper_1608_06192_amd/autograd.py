"""Unrolled Frank-Wolfe as a torch.autograd.Function.

y_T = FW^T(softmax(-phi)) with the QP of Sec. 4 (exact line search of
App. B), differentiable in the unaries phi and the kernel weights w_m. The
forward and the reverse sweep both run in the HIP library (dcrf_fw_forward /
dcrf_fw_backward); this module only marshals tensors.

Memory: the forward keeps, per iteration t, the iterate y_t and
P_t = (Psi + D) y_t (N x L each), the conditional gradient's labels s_t
(N int32), each lattice's blurred vertex values of the one-hot s_t (and of
y_0), and four scalars: about 2 T N L values, 363 MB at 500x375, L = 21,
T = 10 in FP32 (Context.fw_saved_size gives the exact figure). The reverse
sweep reads them and runs no filter inside its loop. With
``recompute=True`` the checkpoint is dropped after the forward and rebuilt
by a second forward at backward time, so that nothing of size T x N x L
stays alive between the two passes (the peak during backward is the same).

On a context that holds a batch of images (``Context.set_images``) the
unaries and marginals are the packed arrays of the batch, every image takes
its own steps, and the shared weights receive the sum of the images'
gradients (summed in the library).
"""

from __future__ import annotations

import torch

from .dcrf import Context


class UnrolledFrankWolfe(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, unary: torch.Tensor, weights: torch.Tensor,
                mu: torch.Tensor, iters: int, recompute: bool = False):
        w = [float(v) for v in weights.detach().cpu().tolist()]
        mu = None if mu is None else mu.contiguous()
        y, saved = ctx.fw_forward(unary.detach().contiguous(), mu, iters, w=w)
        fctx.dcrf = ctx
        fctx.iters = iters
        fctx.recompute = recompute
        fctx.w = w
        fctx.wdtype, fctx.wdevice = weights.dtype, weights.device
        if recompute:
            saved = None
        fctx.save_for_backward(unary.detach().contiguous(), mu)
        fctx.saved_ckpt = saved
        return y

    @staticmethod
    def backward(fctx, grad_y: torch.Tensor):
        unary, mu = fctx.saved_tensors
        ctx: Context = fctx.dcrf
        # the context may have been used with other weights in between
        ctx.set_weights(fctx.w)
        saved = fctx.saved_ckpt
        if saved is None:
            _, saved = ctx.fw_forward(unary, mu, fctx.iters, w=fctx.w)
        gphi, gw = ctx.fw_backward(unary, mu, fctx.iters, saved,
                                   grad_y.contiguous(), summed=True)
        fctx.saved_ckpt = None
        gw_t = torch.tensor(gw, dtype=fctx.wdtype, device=fctx.wdevice)
        return None, gphi, gw_t, None, None, None


def unrolled_frank_wolfe(ctx: Context, unary: torch.Tensor,
                         weights: torch.Tensor, mu: torch.Tensor, iters: int,
                         recompute: bool = False) -> torch.Tensor:
    """y_T after ``iters`` Frank-Wolfe iterations from softmax(-unary) on the
    context's image, with the kernel weights ``weights`` (nk values)."""
    return UnrolledFrankWolfe.apply(ctx, unary, weights, mu, iters, recompute)
