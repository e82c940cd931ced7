"""Differentiable batched FFT with an ABFT-protected, hand-written adjoint.

Forward: y = W x along the last axis (TurboFFT Sec. 2.2, w_N = exp(-2 pi i/N)).
The map is complex-linear, so PyTorch's gradient convention gives
grad_x = W^H grad_y = conj(W) grad_y (W is symmetric): the unnormalised
inverse transform, run by the same fault-tolerant kernels (dir = +1,
scale = 1).  Both directions accumulate into one counters tensor.
"""
from __future__ import annotations

import torch

from . import _lib
from .fft import fft_c2c, new_counts


class FFT(torch.autograd.Function):
    """y = FFT(x) over the last dimension; x is complex64 or complex128 on the GPU."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, ft_mode: int = _lib.FT_CORRECT, counts=None):
        shape = x.shape
        N = shape[-1]
        x2 = x.reshape(-1, N).contiguous()
        if ft_mode != _lib.FT_OFF and counts is None:
            counts = new_counts(x.device)
        y, _ = fft_c2c(x2, dir=_lib.FORWARD, ft_mode=ft_mode, counts=counts)
        ctx.ft_mode = ft_mode
        ctx.counts = counts
        ctx.shape = shape
        return y.reshape(shape)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        N = ctx.shape[-1]
        g2 = g.reshape(-1, N).contiguous()
        gx, _ = fft_c2c(g2, dir=_lib.INVERSE, ft_mode=ctx.ft_mode, counts=ctx.counts, scale=1.0)
        return gx.reshape(ctx.shape), None, None


def fft(x: torch.Tensor, ft_mode: int = _lib.FT_CORRECT, counts=None) -> torch.Tensor:
    """Differentiable forward transform along the last axis."""
    return FFT.apply(x, ft_mode, counts)
