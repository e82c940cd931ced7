"""Python entry points over the C ABI, on torch tensors and torch streams.

    fft_c2c(x, dir=-1, ft_mode=2, out=None, counts=None, scale=0.0) -> (y, counts)

x is a [batch, N] complex64 (fp32) or complex128 (fp64) CUDA tensor.  The
call runs on torch's current stream; counts is a device int64 tensor of 8
entries laid out like tfft_ft_counts (detected, corrected, rebuilt,
uncorrectable, last_signal, calib, sched_errors, fallback), accumulated,
never synchronised.
"""
from __future__ import annotations

import torch

from . import _lib

COUNT_FIELDS = ("detected", "corrected", "rebuilt", "uncorrectable", "last_signal", "calib",
                "sched_errors", "fallback")


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


def fft_c2c_noalloc(x: torch.Tensor, out: torch.Tensor, dir: int = -1, ft_mode: int = 2,
                    counts: torch.Tensor | None = None, scale: float = 0.0):
    """tfft_c2c_noalloc: the transform of fft_c2c without any device
    allocation (two-pass intermediates in the library's static scratch
    array).  out, and counts unless ft_mode is FT_OFF, are supplied by the
    caller; the tables of the length must have been built by prepare()."""
    if not (x.is_cuda and out.is_cuda):
        raise ValueError("x and out must be device tensors")
    if x.dim() != 2 or not x.is_contiguous():
        raise ValueError("x must be a contiguous [batch, N] tensor")
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x in shape, dtype, device and be contiguous")
    if ft_mode != _lib.FT_OFF and counts is None:
        raise ValueError("counts is required unless ft_mode is FT_OFF")
    prec = _precision(x.dtype)
    batch, N = x.shape
    cptr = counts.data_ptr() if counts is not None else None
    with torch.cuda.device(x.device):
        st = _lib.load().tfft_c2c_noalloc(x.data_ptr(), out.data_ptr(), N, batch, dir, prec, ft_mode,
                                          float(scale), cptr, _stream_ptr(x.device))
    _lib.check(st, f"tfft_c2c_noalloc(N={N}, batch={batch}, dir={dir}, ft={ft_mode})")
    return out, counts


def fft_c2c_offline(x: torch.Tensor, dir: int = -1, out: torch.Tensor | None = None,
                    counts: torch.Tensor | None = None, scale: float = 0.0):
    """tfft_c2c_offline: the transform with offline (unfused) two-side ABFT,
    the comparison baseline for the fused kernels."""
    if not x.is_cuda or x.dim() != 2 or not x.is_contiguous():
        raise ValueError("x must be a contiguous [batch, N] device tensor")
    prec = _precision(x.dtype)
    batch, N = x.shape
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x in shape, dtype, device and be contiguous")
    if counts is None:
        counts = new_counts(x.device)
    with torch.cuda.device(x.device):
        st = _lib.load().tfft_c2c_offline(x.data_ptr(), out.data_ptr(), N, batch, dir, prec, float(scale),
                                          counts.data_ptr(), _stream_ptr(x.device))
    _lib.check(st, f"tfft_c2c_offline(N={N}, batch={batch}, dir={dir})")
    return out, counts


def fft_c2c_stepwise(x: torch.Tensor, level: int, dir: int = -1, out: torch.Tensor | None = None):
    """tfft_c2c_stepwise: the plain complex64 transform at a level of the
    stepwise study (0 per-stage radix-2 launches, 1 radix-2 stages in one
    launch, 2 default plans, 3 tuned); out of place."""
    if not x.is_cuda or x.dim() != 2 or not x.is_contiguous() or x.dtype != torch.complex64:
        raise ValueError("x must be a contiguous [batch, N] complex64 device tensor")
    batch, N = x.shape
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x in shape, dtype, device and be contiguous")
    with torch.cuda.device(x.device):
        st = _lib.load().tfft_c2c_stepwise(x.data_ptr(), out.data_ptr(), N, batch, dir, int(level),
                                           _stream_ptr(x.device))
    _lib.check(st, f"tfft_c2c_stepwise(N={N}, batch={batch}, level={level})")
    return out


def prepare(N: int, dtype=torch.complex64, ft_mode: int = 2, batch: int = 0, device=None) -> None:
    """Build the tables of length N and, for batch > 0, reserve the two-pass
    workspace for up to `batch` signals on torch's current stream (call
    before capturing fft_c2c into a graph)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        st = _lib.load().tfft_prepare(N, int(batch), _precision(dtype), ft_mode,
                                      _stream_ptr(dev) if batch > 0 else None)
    _lib.check(st, f"tfft_prepare(N={N}, batch={batch})")


def supported(N: int, dtype=torch.complex64) -> bool:
    return bool(_lib.load().tfft_supported(N, _precision(dtype)))


def inject_arm(signal: int, element: int, part: int, bit: int, dtype=torch.complex64,
               pass_: int = -1, stage: int = -1, signal2: int | None = None) -> None:
    """Arm one bit flip for the next call (see tfft_inject_arm_desc): pass_
    -1 last, 0 single / column pass, 1 row pass; stage -1 after the last
    radix stage, else after radix stage `stage`; signal2: the same flip in a
    second signal (two faults in one call)."""
    import ctypes
    d = _lib.InjectDesc(signal=int(signal), element=int(element), part=int(part), bit=int(bit),
                        precision=_precision(dtype), pass_=int(pass_), stage=int(stage),
                        two=0 if signal2 is None else 1, signal2=-1 if signal2 is None else int(signal2))
    _lib.check(_lib.load().tfft_inject_arm_desc(ctypes.byref(d)), "tfft_inject_arm_desc")


def route_info(N: int, dtype=torch.complex64, ft_mode: int = 2) -> dict:
    """The route a call takes now: passes, N1, N2, N3, stages of each pass,
    T, granularity and sub-signals per workgroup of each pass."""
    import ctypes
    buf = (ctypes.c_longlong * 12)()
    _lib.check(_lib.load().tfft_route_info(N, _precision(dtype), ft_mode, buf, 12), f"tfft_route_info(N={N})")
    keys = ("passes", "N1", "N2", "stages0", "stages1", "T", "gran", "slots0", "slots1",
            "N3", "stages2", "slots2")
    return {k: int(buf[i]) for i, k in enumerate(keys)}


def inject_disarm() -> None:
    _lib.load().tfft_inject_disarm()


def set_tuning(N: int, dtype, T: int = 0, kappa: float = 0.0) -> None:
    _lib.check(_lib.load().tfft_set_tuning(N, _precision(dtype), T, float(kappa)), "tfft_set_tuning")


def set_granularity(N: int, dtype, gran: int) -> None:
    """Detection granularity of (N, dtype): 0 once per group (location code),
    1 per transaction (see tfft_set_granularity)."""
    _lib.check(_lib.load().tfft_set_granularity(N, _precision(dtype), int(gran)), "tfft_set_granularity")


def get_tuning(N: int, dtype):
    import ctypes
    T = ctypes.c_int()
    k = ctypes.c_double()
    _lib.check(_lib.load().tfft_get_tuning(N, _precision(dtype), ctypes.byref(T), ctypes.byref(k)),
               "tfft_get_tuning")
    return T.value, k.value


# ---- ragged batches ----
RAGGED_PERSISTENT = 0
RAGGED_PER_SIZE = 1
_MODES = {"persistent": RAGGED_PERSISTENT, "per_size": RAGGED_PER_SIZE}


def ragged_set_schedule(window_elems: int = 0, item_elems: int = 0, waves: int = 3) -> None:
    """Schedule of ragged plans created afterwards (see tfft_ragged_set_schedule)."""
    _lib.check(_lib.load().tfft_ragged_set_schedule(int(window_elems), int(item_elems), int(waves)),
               "tfft_ragged_set_schedule")


def ragged_supported(N: int, dtype=torch.complex64) -> bool:
    return bool(_lib.load().tfft_ragged_supported(N, _precision(dtype)))


class RaggedPlan:
    """A ragged batch: signals of lengths `sizes` packed back to back.

    Built once (allocates device memory, outside any graph capture); each call
    runs the whole batch either as one persistent launch ("persistent") or as
    one launch per length and pass ("per_size"), on torch's current stream.
    """

    def __init__(self, sizes, dtype=torch.complex64, device=None):
        import ctypes
        self.sizes = [int(n) for n in sizes]
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        arr = (ctypes.c_longlong * max(1, len(self.sizes)))(*self.sizes)
        h = ctypes.c_void_p()
        lib = _lib.load()
        with torch.cuda.device(self.device):
            st = lib.tfft_ragged_plan_create(ctypes.byref(h), arr, len(self.sizes), _precision(dtype))
        _lib.check(st, f"tfft_ragged_plan_create({len(self.sizes)} signals)")
        self._h = h
        self.total = sum(self.sizes)
        self.offsets = [0]
        for n in self.sizes:
            self.offsets.append(self.offsets[-1] + n)

    def info(self, device_state: bool = False) -> dict:
        import ctypes
        n = 10 if device_state else 8
        buf = (ctypes.c_longlong * 10)()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().tfft_ragged_plan_info(self._h, buf, n), "tfft_ragged_plan_info")
        keys = ("signals", "total", "items", "classes", "ws_elems", "grid", "batches", "window",
                "err_launches", "queue_next")
        return {k: int(buf[i]) for i, k in enumerate(keys[:n])}

    def __call__(self, x: torch.Tensor, out: torch.Tensor | None = None, dir: int = -1,
                 ft_mode: int = 2, counts: torch.Tensor | None = None, unit_scale: bool = False,
                 mode: str = "persistent"):
        if self._h is None:
            raise RuntimeError("plan was closed")
        if not x.is_cuda or x.dtype != self.dtype or not x.is_contiguous() or x.numel() != self.total:
            raise ValueError(f"x must be a contiguous {self.dtype} device tensor of {self.total} elements")
        if out is None:
            out = torch.empty_like(x)
        elif out.dtype != x.dtype or not out.is_contiguous() or out.numel() != self.total or out.device != x.device:
            raise ValueError("out must match x")
        if ft_mode != _lib.FT_OFF and counts is None:
            counts = new_counts(x.device)
        cptr = counts.data_ptr() if counts is not None else None
        with torch.cuda.device(x.device):
            st = _lib.load().tfft_c2c_ragged(self._h, x.data_ptr(), out.data_ptr(), dir,
                                             1 if unit_scale else 0, _MODES[mode], ft_mode, cptr,
                                             _stream_ptr(x.device))
        _lib.check(st, f"tfft_c2c_ragged({len(self.sizes)} signals, mode={mode}, ft={ft_mode})")
        return out, counts

    def split(self, packed: torch.Tensor) -> list:
        return [packed[self.offsets[i]:self.offsets[i + 1]] for i in range(len(self.sizes))]

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            with torch.cuda.device(self.device):
                _lib.load().tfft_ragged_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ragged_cache: dict = {}


def fft_c2c_ragged(packed: torch.Tensor, sizes, dir: int = -1, ft_mode: int = 2,
                   out: torch.Tensor | None = None, counts: torch.Tensor | None = None,
                   mode: str = "persistent"):
    """Transform the signals of lengths `sizes` packed back to back in `packed`.

    Plans are cached per (device, sizes); the first call for a list builds it.
    """
    key = (str(packed.device), packed.dtype, tuple(int(n) for n in sizes))
    plan = _ragged_cache.get(key)
    if plan is None:
        plan = RaggedPlan(key[2], dtype=packed.dtype, device=packed.device)
        _ragged_cache[key] = plan
    return plan(packed, out=out, dir=dir, ft_mode=ft_mode, counts=counts, mode=mode)


# ---- routes and the tuning table ----
def route_code(n1: int, variant_a: int = 0, variant_b: int = 0, n2: int = 0) -> int:
    """Route code: n1 = 1 single pass (plan variant_a), n1 > 1 column pass of n1
    points (variant_a) then row pass of N/n1 (variant_b); with n2 (a power of
    two) the three passes n1, n2, N/(n1 n2)."""
    lg = int(n2).bit_length() - 1 if n2 else 0
    return int(n1) | (int(variant_a) << 32) | (int(variant_b) << 40) | (lg << 48)


def route_parts(code: int):
    """(n1, variant_a, variant_b) of a route code."""
    return code & 0xFFFFFFFF, (code >> 32) & 0xFF, (code >> 40) & 0xFF


def route_n2(code: int) -> int:
    """The second length of a three-pass route code (0 below three passes)."""
    lg = (code >> 48) & 0x3F
    return 1 << lg if lg else 0


def routes(N: int, dtype=torch.complex64, ft_mode: int = 2) -> list:
    """Route codes built for length N (see route_code)."""
    import ctypes
    lib = _lib.load()
    n = lib.tfft_routes(N, _precision(dtype), ft_mode, None, 0)
    _lib.check(min(n, 0), f"tfft_routes(N={N})")
    buf = (ctypes.c_longlong * max(1, n))()
    lib.tfft_routes(N, _precision(dtype), ft_mode, buf, n)
    return [int(buf[i]) for i in range(n)]


def set_route(N: int, dtype, code: int) -> None:
    """Fix the route of length N in every ABFT mode (0: the default policy)."""
    _lib.check(_lib.load().tfft_set_route(N, _precision(dtype), code), f"tfft_set_route(N={N})")


def get_route(N: int, dtype=torch.complex64, ft_mode: int = 2) -> int:
    import ctypes
    v = ctypes.c_longlong()
    _lib.check(_lib.load().tfft_get_route(N, _precision(dtype), ft_mode, ctypes.byref(v)),
               f"tfft_get_route(N={N})")
    return int(v.value)


def set_chunk(N: int, dtype, chunk_bytes: int) -> None:
    _lib.check(_lib.load().tfft_set_chunk(N, _precision(dtype), chunk_bytes), f"tfft_set_chunk(N={N})")


def load_tuning(path: str) -> int:
    """Apply a tuning table written by the autotuner; returns the entries applied."""
    n = _lib.load().tfft_load_tuning(str(path).encode())
    _lib.check(min(n, 0), f"tfft_load_tuning({path})")
    return n
