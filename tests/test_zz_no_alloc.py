"""tfft_c2c_noalloc: the transform of tfft_c2c without any device allocation.

Two-pass lengths keep their intermediate in the library's static per-device
scratch array (64 MiB), in chunks of whole signals that fit it.  Checked
against tfft_c2c on the same inputs (bit for bit when no fault is injected,
since every signal's transform is independent of how the batch is chunked)
and against the oracle on sampled signals, on two calls in a row, the second
with a smaller input.
"""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")
from paper_2412_05824_amd import _lib  # noqa: E402

TOL = {torch.complex64: 2e-6, torch.complex128: 1e-13}
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _noalloc(x, y, dir, ft_mode, counts):
    """Call the C entry point itself (argument marshalling only)."""
    batch, N = x.shape
    prec = _lib.FP32 if x.dtype == torch.complex64 else _lib.FP64
    st = _lib.load().tfft_c2c_noalloc(x.data_ptr(), y.data_ptr(), N, batch, dir, prec, ft_mode, 0.0,
                                      counts.data_ptr() if counts is not None else None,
                                      torch.cuda.current_stream(x.device).cuda_stream)
    assert st == _lib.TFFT_OK, _lib.strerror(st)


def _case(dev, N, batch, dtype, dir, ft_mode, seed, inplace=False):
    npdt = np.complex64 if dtype == torch.complex64 else np.complex128
    xh = synth.signals(batch, N, seed=seed, dtype=npdt)
    x = torch.from_numpy(xh).to(dev)
    tf.prepare(N, dtype, ft_mode)                  # tables only: allocates, before the call
    ref_y, ref_c = tf.fft_c2c(x.clone(), dir=dir, ft_mode=ft_mode)
    y = x.clone() if inplace else torch.empty_like(x)
    counts = tf.new_counts(dev)
    torch.cuda.synchronize()
    _noalloc(y if inplace else x, y, dir, ft_mode, counts if ft_mode else None)
    torch.cuda.synchronize()
    assert torch.equal(y, ref_y), (N, batch)
    if ft_mode:
        c = tf.counts_dict(counts)
        assert c["detected"] == 0 and tf.counts_dict(ref_c)["detected"] == 0, c
    pick = sorted({0, batch // 2, batch - 1})
    ref = oracle.fft(xh[pick], dir=dir, threads=8)
    got = y[pick].cpu().numpy()
    for i in range(len(pick)):
        assert oracle.rel_l2(got[i], ref[i]) <= TOL[dtype], (N, pick[i])


@pytest.mark.parametrize("first,second", [
    # fp32 2^20: 8 MiB per signal, 8 per scratch chunk, 20 signals = 3 chunks;
    # then a smaller two-pass call that fits one chunk
    ((1 << 20, 20, torch.complex64, -1, 2), (1 << 14, 10, torch.complex64, -1, 2)),
    # fp64 2^20 inverse (16 MiB per signal, 4 per chunk), then a single pass
    ((1 << 20, 9, torch.complex128, 1, 2), (4096, 7, torch.complex128, -1, 0)),
    # the largest fp32 length (32 MiB per signal, 2 per chunk), then 2^16
    ((1 << 22, 5, torch.complex64, -1, 0), (1 << 16, 3, torch.complex64, 1, 1)),
])
def test_noalloc_matches_c2c_two_calls(dev, first, second):
    for k, (N, batch, dtype, dir, ft) in enumerate((first, second)):
        _case(dev, N, batch, dtype, dir, ft, seed=9100 + 10 * k + N % 97)


def test_noalloc_in_place_single_pass(dev):
    _case(dev, 4096, 33, torch.complex64, -1, 2, seed=9150, inplace=True)
    _case(dev, 256, 17, torch.complex64, -1, 2, seed=9151, inplace=True)


def test_noalloc_corrects_column_pass_flip(dev):
    """A flip in the column pass (its result sits in the scratch array) is
    detected, located and corrected within the tolerance of the fault-free
    output of tfft_c2c; a second, smaller call after it is clean."""
    N, batch = 1 << 22, 5
    xh = synth.signals(batch, N, seed=9160)
    x = torch.from_numpy(xh).to(dev)
    tf.prepare(N, torch.complex64, 2)
    clean, _ = tf.fft_c2c(x, ft_mode=2)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    info = tf.route_info(N, torch.complex64, 2)
    assert info["passes"] == 2
    tf.inject_arm(signal=3, element=12345, part=1, bit=28, dtype=torch.complex64, pass_=0, stage=-1)
    _noalloc(x, y, -1, 2, counts)
    torch.cuda.synchronize()
    c = tf.counts_dict(counts)
    assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == 3, c
    for b in range(batch):
        d = oracle.rel_l2(y[b].cpu().numpy(), clean[b].cpu().numpy())
        assert d <= TOL[torch.complex64], (b, d)
        if b != 3:
            assert torch.equal(y[b], clean[b]), b
    _case(dev, 1 << 16, 6, torch.complex64, -1, 2, seed=9161)


def test_noalloc_refuses_unprepared_length(dev):
    """In a fresh process, a length whose tables were never built is refused
    with TFFT_ENOTPREPARED (nothing launched), then runs once prepared."""
    code = (
        "import sys, torch; sys.path.insert(0, %r)\n"
        "from paper_2412_05824_amd import _lib\n"
        "import paper_2412_05824_amd as tf\n"
        "x = torch.zeros(4, 1 << 18, dtype=torch.complex128, device='cuda:0'); y = torch.empty_like(x)\n"
        "st = torch.cuda.current_stream().cuda_stream\n"
        "r1 = _lib.load().tfft_c2c_noalloc(x.data_ptr(), y.data_ptr(), 1 << 18, 4, -1, 1, 0, 0.0, None, st)\n"
        "tf.prepare(1 << 18, torch.complex128, 0)\n"
        "r2 = _lib.load().tfft_c2c_noalloc(x.data_ptr(), y.data_ptr(), 1 << 18, 4, -1, 1, 0, 0.0, None, st)\n"
        "torch.cuda.synchronize(); ok = bool((y == 0).all())\n"
        "print('STATUS', r1, r2, ok, flush=True)\n" % ROOT)
    print("noalloc unprepared-length child process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("STATUS")][-1]
    assert line.split()[1:] == [str(_lib.TFFT_ENOTPREPARED), str(_lib.TFFT_OK), "True"], line
