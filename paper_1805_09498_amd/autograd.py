"""Differentiable unrolled FastFCA-AS for PyTorch.

``unrolled_separate(x, v0, lam0, P0, n_iter, ckpt_every)`` runs n_iter hybrid
iterations (Section 4.3 of the paper) from (v0, lam0, P0) and returns the
Wiener estimates of the sources (eq. 3 with eq. 15), [J][F][N][I] complex64.
Its backward pass is the library's hand-written adjoint
(``fastfca_as_backward``): gradients reach x, v0, lam0 and P0, and the
iterations are recomputed from a checkpoint every ``ckpt_every`` iterations
instead of being stored.  The complex-gradient convention is PyTorch's
(dL/dRe z + i dL/dIm z for a real loss), which is also the library's.
"""

import torch

from . import fastfca as ff


class UnrolledFastFCA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, v0, lam0, P0, n_iter, ckpt_every):
        c = ff.fca_init(ff.FCA_METHOD_AS, x.detach().contiguous(), v0.detach().contiguous(),
                        lam0.detach().contiguous(), P0.detach().contiguous())
        out = ff.fastfca_as_forward(c, n_iter, ckpt_every)
        ctx.fca = c
        return out

    @staticmethod
    def backward(ctx, grad_out):
        need = tuple(bool(n) for n in ctx.needs_input_grad[:4])
        gx, gv, gl, gP = ff.fastfca_as_backward(ctx.fca, grad_out.contiguous(), need)
        return gx, gv, gl, gP, None, None


def unrolled_separate(x, v0, lam0, P0, n_iter=20, ckpt_every=5):
    """x [F][N][I] complex64, v0 [F][N][J] float32, lam0 [F][J][I] float32,
    P0 [F][I][I] complex64, all on the GPU.  Returns [J][F][N][I] complex64."""
    return UnrolledFastFCA.apply(x, v0, lam0, P0, int(n_iter), int(ckpt_every))
