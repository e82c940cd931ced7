"""CPU fp64 oracle for the batched C2C DFT -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2412_05824_amd``) and never imports it.

Definitions followed (TurboFFT, Sec. 2.2 "DFT and FFT"):
  forward  y_k = sum_n x_n exp(-2 pi i k n / N)          (dir = -1, scale 1)
  inverse  x_k = (1/N) sum_n y_n exp(+2 pi i k n / N)    (dir = +1, scale 1/N)

``fft`` runs the recursive radix-2/3 factorisation in plain C (fp64),
``dft`` the O(N^2) matrix-vector product, ``dft_bins`` single output bins.
Inputs of any complex dtype are upcast exactly to complex128.
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_twiddle.argtypes = [ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int, dp, dp]
    lib.oracle_twiddle.restype = None
    lib.oracle_dft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int]
    lib.oracle_dft.restype = None
    lib.oracle_fft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int]
    lib.oracle_fft.restype = None
    lib.oracle_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                                 ctypes.c_longlong, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_batch.restype = None
    lib.oracle_dft_bins.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                                    ctypes.c_longlong, ctypes.c_int, ctypes.c_void_p]
    lib.oracle_dft_bins.restype = None
    _lib = lib
    return lib


def twiddle(N: int, m: int, sign: int) -> complex:
    """exp(sign * 2 pi i m / N), accurately reduced (Sec. 2.2)."""
    lib = _load()
    re, im = ctypes.c_double(), ctypes.c_double()
    lib.oracle_twiddle(N, m, sign, ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def _as_c128(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x), dtype=np.complex128)
    return a


def _run_batch(x2: np.ndarray, N: int, dir: int, scale: float, use_dft: bool, threads: int):
    count = x2.shape[0]
    y2 = np.empty_like(x2)
    lib = _load()
    if count == 0:
        return y2
    threads = max(1, min(threads, count))
    chunks = np.array_split(np.arange(count), threads)

    def work(idx):
        if len(idx) == 0:
            return
        lo, hi = int(idx[0]), int(idx[-1]) + 1
        xs = x2[lo:hi]
        ys = y2[lo:hi]
        lib.oracle_batch(xs.ctypes.data, ys.ctypes.data, N, hi - lo, dir, scale, int(use_dft))

    if threads == 1:
        work(chunks[0])
    else:  # ctypes drops the GIL for the duration of each C call
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, chunks))
    return y2


def fft(x, dir: int = -1, scale: float | None = None, threads: int = 1) -> np.ndarray:
    """Transform along the last axis with the recursive factorisation.

    dir = -1 forward (scale defaults to 1), dir = +1 inverse (scale defaults
    to 1/N).  Returns complex128 of x's shape.
    """
    a = _as_c128(x)
    N = a.shape[-1]
    if scale is None:
        scale = 1.0 if dir == -1 else 1.0 / N
    y = _run_batch(a.reshape(-1, N), N, dir, float(scale), False, threads)
    return y.reshape(a.shape)


def dft(x, dir: int = -1, scale: float | None = None, threads: int = 1) -> np.ndarray:
    """Same as ``fft`` but with the O(N^2) matrix-vector product."""
    a = _as_c128(x)
    N = a.shape[-1]
    if scale is None:
        scale = 1.0 if dir == -1 else 1.0 / N
    y = _run_batch(a.reshape(-1, N), N, dir, float(scale), True, threads)
    return y.reshape(a.shape)


def dft_bins(x, ks, dir: int = -1) -> np.ndarray:
    """Output bins y_k (k in ks) of one signal x, O(N) each, unscaled."""
    a = _as_c128(x).reshape(-1)
    k = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    out = np.empty(k.shape[0], dtype=np.complex128)
    _load().oracle_dft_bins(a.ctypes.data, a.shape[0], k.ctypes.data, k.shape[0], dir,
                            out.ctypes.data)
    return out


def rel_l2(got, ref) -> float:
    """||got - ref||_2 / ||ref||_2 in fp64 (the acceptance metric)."""
    g = np.asarray(got, dtype=np.complex128)
    r = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(r.ravel())
    num = np.linalg.norm((g - r).ravel())
    return float(num / den) if den > 0 else float(num)
