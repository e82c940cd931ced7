"""Python entry points over the C ABI, on torch tensors and torch streams.

    fft_c2c(x, dir=-1, ft_mode=2, out=None, counts=None, scale=0.0) -> (y, counts)

x is a [batch, N] complex64 (fp32) or complex128 (fp64) CUDA tensor.  The
call runs on torch's current stream; counts is a device int64 tensor of 8
entries laid out like tfft_ft_counts (detected, corrected, rebuilt,
uncorrectable, last_signal, reserved...), accumulated, never synchronised.
"""
from __future__ import annotations

import torch

from . import _lib

COUNT_FIELDS = ("detected", "corrected", "rebuilt", "uncorrectable", "last_signal")


def _precision(dtype) -> int:
    if dtype == torch.complex64:
        return _lib.FP32
    if dtype == torch.complex128:
        return _lib.FP64
    raise TypeError(f"unsupported dtype {dtype}: use complex64 or complex128")


def new_counts(device) -> torch.Tensor:
    return torch.zeros(8, dtype=torch.int64, device=device)


def counts_dict(counts: torch.Tensor) -> dict:
    c = counts.detach().cpu().tolist()
    return {k: int(c[i]) for i, k in enumerate(COUNT_FIELDS)}


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def fft_c2c(x: torch.Tensor, dir: int = -1, ft_mode: int = 2, out: torch.Tensor | None = None,
            counts: torch.Tensor | None = None, scale: float = 0.0):
    if not x.is_cuda:
        raise ValueError("x must be a device tensor")
    if x.dim() != 2:
        raise ValueError("x must be [batch, N]")
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    prec = _precision(x.dtype)
    batch, N = x.shape
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x in shape, dtype, device and be contiguous")
    if ft_mode != _lib.FT_OFF and counts is None:
        counts = new_counts(x.device)
    cptr = counts.data_ptr() if counts is not None else None
    with torch.cuda.device(x.device):
        st = _lib.load().tfft_c2c(x.data_ptr(), out.data_ptr(), N, batch, dir, prec, ft_mode,
                                  float(scale), cptr, _stream_ptr(x.device))
    _lib.check(st, f"tfft_c2c(N={N}, batch={batch}, dir={dir}, ft={ft_mode})")
    return out, counts


def prepare(N: int, dtype=torch.complex64, ft_mode: int = 2) -> None:
    _lib.check(_lib.load().tfft_prepare(N, _precision(dtype), ft_mode), f"tfft_prepare(N={N})")


def supported(N: int, dtype=torch.complex64) -> bool:
    return bool(_lib.load().tfft_supported(N, _precision(dtype)))


def inject_arm(signal: int, element: int, part: int, bit: int, dtype=torch.complex64) -> None:
    _lib.check(_lib.load().tfft_inject_arm(signal, element, part, bit, _precision(dtype)),
               "tfft_inject_arm")


def inject_disarm() -> None:
    _lib.load().tfft_inject_disarm()


def set_tuning(N: int, dtype, T: int = 0, kappa: float = 0.0) -> None:
    _lib.check(_lib.load().tfft_set_tuning(N, _precision(dtype), T, float(kappa)), "tfft_set_tuning")


def get_tuning(N: int, dtype):
    import ctypes
    T = ctypes.c_int()
    k = ctypes.c_double()
    _lib.check(_lib.load().tfft_get_tuning(N, _precision(dtype), ctypes.byref(T), ctypes.byref(k)),
               "tfft_get_tuning")
    return T.value, k.value
