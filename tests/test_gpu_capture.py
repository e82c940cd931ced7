"""Graph capture of the uniform path (tfft_c2c) and its workspace contract.

A two-pass length needs the library's workspace.  Reserved beforehand with
tfft_prepare(N, batch, ..., stream), a call captured on that stream
allocates nothing; a later, larger eager call on the same stream grows the
workspace without freeing the captured buffer, so replays stay correct.
Replays run with new data and eager work in between, each checked against
the eager result and the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_capture_two_pass_then_larger_eager_call(dev):
    N, batch = 1 << 14, 48
    s = torch.cuda.Stream(device=dev)
    x = torch.empty(batch, N, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    with torch.cuda.stream(s):
        tf.prepare(N, torch.complex64, tf.FT_CORRECT, batch=batch)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tf.fft_c2c(x, ft_mode=tf.FT_CORRECT, out=y, counts=counts)
    torch.cuda.synchronize()
    big_n, big_batch = 1 << 20, 96
    xb = torch.from_numpy(synth.signals(big_batch, big_n, seed=8101)).to(dev)
    for r in range(3):
        fresh = synth.signals(batch, N, seed=8200 + r)
        x.copy_(torch.from_numpy(fresh).to(dev))
        # eager work on the capture stream: the larger length grows the workspace
        with torch.cuda.stream(s):
            yb, cb = tf.fft_c2c(xb, ft_mode=tf.FT_CORRECT)
            eager, _ = tf.fft_c2c(x, ft_mode=tf.FT_CORRECT)
        torch.cuda.synchronize()
        counts.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), r
        assert tf.counts_dict(counts)["detected"] == 0
        assert tf.counts_dict(cb)["detected"] == 0
        pick = [0, batch // 2, batch - 1]
        ref = oracle.fft(fresh[pick], threads=8)
        got = y.cpu().numpy()[pick]
        assert oracle.rel_l2(got, ref) <= 2e-6, r
    refb = oracle.fft(xb[[0, big_batch - 1]].cpu().numpy(), threads=8)
    assert oracle.rel_l2(yb[[0, big_batch - 1]].cpu().numpy(), refb) <= 2e-6


def test_capture_without_reservation_is_refused(dev):
    """A two-pass call captured on a stream that never had a workspace would
    have to allocate: it returns TFFT_ECAPTURE instead (the capture is then
    abandoned by torch)."""
    N = 1 << 15
    s = torch.cuda.Stream(device=dev)
    x = torch.zeros(4, N, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    tf.prepare(N, torch.complex64, tf.FT_OFF)   # tables only, no workspace
    g = torch.cuda.CUDAGraph()
    with pytest.raises(tf.TfftError) as ei:
        with torch.cuda.graph(g, stream=s):
            tf.fft_c2c(x, ft_mode=tf.FT_OFF, out=y)
    assert ei.value.status == -6
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 4096), (torch.complex128, 1 << 16)])
def test_capture_replays_match_eager(dev, dtype, N):
    batch = 24
    npdt = np.complex64 if dtype == torch.complex64 else np.complex128
    s = torch.cuda.Stream(device=dev)
    x = torch.empty(batch, N, dtype=dtype, device=dev)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    with torch.cuda.stream(s):
        tf.prepare(N, dtype, tf.FT_CORRECT, batch=batch)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tf.fft_c2c(x, ft_mode=tf.FT_CORRECT, out=y, counts=counts)
        tf.fft_c2c(y, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT, out=y, counts=counts)
    for r in range(3):
        fresh = synth.signals(batch, N, seed=8300 + r, dtype=npdt)
        x.copy_(torch.from_numpy(fresh).to(dev))
        e1, _ = tf.fft_c2c(x, ft_mode=tf.FT_CORRECT)
        e2, _ = tf.fft_c2c(e1, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT)
        torch.cuda.synchronize()
        counts.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, e2), r
        assert tf.counts_dict(counts)["detected"] == 0
