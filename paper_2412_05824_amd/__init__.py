"""MI355X-native batched C2C FFT with fused two-side ABFT (TurboFFT method).

The transform runs in hand-written HIP kernels (libtfft.so, gfx950) behind the
C ABI of include/tfft.h; this package is a thin binding over it.
"""
from ._lib import (FORWARD, INVERSE, FP32, FP64, FT_OFF, FT_DETECT, FT_CORRECT, FT_THREAD,  # noqa: F401
                   TfftError)
from .fft import (fft_c2c, fft_c2c_noalloc, fft_c2c_offline, fft_c2c_stepwise, prepare, supported, inject_arm, inject_disarm, route_info,  # noqa: F401
                  set_tuning, set_granularity, get_tuning, new_counts, counts_dict, RaggedPlan, fft_c2c_ragged,
                  ragged_supported, ragged_set_schedule, RAGGED_PERSISTENT, RAGGED_PER_SIZE, routes, route_code, route_parts, route_n2, set_route,
                  get_route, set_chunk, load_tuning)
from .autograd import FFT, fft  # noqa: F401,E402
from . import _lib  # noqa: E402,F401
