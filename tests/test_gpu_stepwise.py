"""The stepwise levels of the plain transform (Sec. 5.1, v0..v3) compute the
same DFT: each level against the CPU fp64 oracle, forward and inverse,
relative L2 <= 2e-6 per signal (fp32), through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = 2e-6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _per_signal_rel(got, ref):
    return np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)


@pytest.mark.parametrize("N", [64, 256, 2048, 4096, 8192, 1 << 16, 1 << 20])
def test_levels_match_oracle(dev, N):
    batch = max(3, (1 << 18) // N) + 1
    x = synth.signals(batch, N, seed=8800 + N)
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, threads=8)
    refi = oracle.fft(x, dir=1, threads=8)
    for level in (0, 1, 2, 3):
        if level == 1 and N > 8192:
            with pytest.raises(RuntimeError):
                tf.fft_c2c_stepwise(xd, level)
            continue
        y = tf.fft_c2c_stepwise(xd, level)
        rel = _per_signal_rel(y.cpu().numpy(), ref)
        assert rel.max() <= TOL, (N, level, rel.max())
        yi = tf.fft_c2c_stepwise(xd, level, dir=tf.INVERSE)
        rel = _per_signal_rel(yi.cpu().numpy(), refi)
        assert rel.max() <= TOL, (N, level, "inverse", rel.max())


def test_level3_equals_plain_library_call(dev):
    N = 1 << 14
    x = synth.signals(9, N, seed=8899)
    xd = torch.from_numpy(x).to(dev)
    y3 = tf.fft_c2c_stepwise(xd, 3)
    y, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    assert torch.equal(y, y3)


def test_in_place_refused(dev):
    xd = torch.zeros(2, 256, dtype=torch.complex64, device=dev)
    with pytest.raises(RuntimeError):
        tf.fft_c2c_stepwise(xd, 0, out=xd)
