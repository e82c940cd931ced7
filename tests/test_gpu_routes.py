"""GPU parity of every route the autotuner may choose.

A length runs single pass or as a column pass of n1 points and a row pass of
N/n1 (Sec. 3.1); the tuning table may pick any built route, any group size T
within the accuracy bound and any chunk.  Each forced choice must reproduce
the oracle within the acceptance tolerance (2e-6 fp32, 1e-13 fp64 relative
L2 per signal) and count no detection on fault-free data.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = {torch.complex64: 2e-6, torch.complex128: 1e-13}
NPDT = {torch.complex64: np.complex64, torch.complex128: np.complex128}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check(dev, dtype, N, batch, seed):
    x_host = synth.signals(batch, N, seed=seed, dtype=NPDT[dtype])
    x = torch.from_numpy(x_host).to(dev)
    y, counts = tf.fft_c2c(x, ft_mode=tf.FT_CORRECT)
    torch.cuda.synchronize()
    assert tf.counts_dict(counts)["detected"] == 0
    # every element: the checksums must not disturb what the plan stores
    y0, _ = tf.fft_c2c(x, ft_mode=tf.FT_OFF)
    assert torch.equal(y, y0), (N, "ABFT and plain outputs differ")
    pick = synth.sample_indices(batch, 6, seed=seed + 1)
    ref = oracle.fft(x_host[pick], threads=8)
    got = y.cpu().numpy()[pick]
    for i in range(len(pick)):
        e = oracle.rel_l2(got[i], ref[i])
        assert e <= TOL[dtype], (N, int(pick[i]), e)


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 1 << 12), (torch.complex64, 1 << 13), (torch.complex64, 1 << 14),
                                     (torch.complex64, 1 << 17), (torch.complex64, 1 << 20),
                                     (torch.complex128, 1 << 11), (torch.complex128, 1 << 16)])
def test_every_route_matches_oracle(dev, dtype, N):
    routes = tf.routes(N, dtype)
    assert routes, N
    T0, k0 = tf.get_tuning(N, dtype)
    try:
        for code in routes:
            n1 = tf.route_parts(code)[0]
            tf.set_route(N, dtype, code)
            assert tf.get_route(N, dtype) == code
            # two chunks at least on the two-pass routes, with a ragged last one
            if n1 > 1:
                tf.set_chunk(N, dtype, max(N * (16 if dtype == torch.complex128 else 8) * 3, 1 << 20))
            batch = max(5, (1 << 21) // N) + 1
            _check(dev, dtype, N, batch, seed=N + n1 + (code >> 32))
    finally:
        tf.set_route(N, dtype, 0)
        tf.set_tuning(N, dtype, T0, k0)
        tf.set_chunk(N, dtype, 128 << 20)
        # back to the package's tuning table for this length
        import os
        if os.path.exists(tf._lib.TUNING_PATH):
            tf.load_tuning(tf._lib.TUNING_PATH)


@pytest.mark.parametrize("T", [1, 2, 4, 8, 16])
def test_group_sizes_fp64(dev, T):
    N = 1024
    T0, k0 = tf.get_tuning(N, torch.complex128)
    try:
        tf.set_tuning(N, torch.complex128, T, 0)
        _check(dev, torch.complex128, N, 16 * T + 3, seed=77 + T)
    finally:
        tf.set_tuning(N, torch.complex128, T0, k0)
