"""Parity at the benchmark's sizes, in the benchmark's launch configuration.

Config "fp32 sweep": complex64, N = 2^6 .. 2^22, batch = 2^27 / N (1 GiB per
buffer), re/im U[-1, 1).  Config "fp64 sweep": complex128, N = 2^6 .. 2^20,
batch = 2^26 / N (1 GiB), re/im N(0, 1), forward then inverse.  Each length
runs its whole batch through the tuned route with two-side ABFT on (the
chunking and the two-level inter-pass twiddles of that length included), as
the benchmark does; a seeded sample of signals (all of them when the batch
holds fewer than 64) is compared one by one with the fp64 oracle at the
acceptance tolerance (relative L2 <= 2e-6 fp32, <= 1e-13 fp64, Sec. 2.2
definition), forward and inverse, and the fault-free batch must count no
detection.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = {torch.complex64: 2e-6, torch.complex128: 1e-13}
CASES = ([(torch.complex64, 1 << k) for k in range(6, 23)] +
         [(torch.complex128, 1 << k) for k in range(6, 21)])


def _id(v):
    if v is torch.complex64:
        return "fp32"
    if v is torch.complex128:
        return "fp64"
    return f"2^{int(v).bit_length() - 1}"


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _per_signal_rel(got, ref):
    return np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)


@pytest.mark.parametrize("dtype,N", CASES, ids=[f"{_id(d)}-{_id(n)}" for d, n in CASES])
def test_full_size_sampled_parity(dev, dtype, N):
    fp32 = dtype == torch.complex64
    total = (1 << 27) if fp32 else (1 << 26)
    batch = total // N
    rdt = torch.float32 if fp32 else torch.float64
    g = torch.Generator(device=dev)
    g.manual_seed(7000 + N + (0 if fp32 else 1))
    if fp32:
        x = torch.rand(total, 2, dtype=rdt, device=dev, generator=g) * 2 - 1
    else:
        x = torch.randn(total, 2, dtype=rdt, device=dev, generator=g)
    x = x.view(dtype).view(batch, N)
    counts = tf.new_counts(dev)
    y, _ = tf.fft_c2c(x, dir=tf.FORWARD, ft_mode=tf.FT_CORRECT, counts=counts)
    yi, _ = tf.fft_c2c(x, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT, counts=counts)
    c = tf.counts_dict(counts)
    assert c["detected"] == 0 and c["uncorrectable"] == 0, c
    n_pick = min(batch, max(64, (1 << 20) // N))
    pick = synth.sample_indices(batch, n_pick, seed=N)
    idx = torch.from_numpy(pick).to(dev)
    xs = x.index_select(0, idx).cpu().numpy()
    ys = y.index_select(0, idx).cpu().numpy()
    yis = yi.index_select(0, idx).cpu().numpy()
    del x, y, yi
    ref = oracle.fft(xs, dir=-1, threads=16)
    per = _per_signal_rel(ys, ref)
    assert per.max() <= TOL[dtype], (N, int(pick[per.argmax()]), per.max())
    refi = oracle.fft(xs, dir=+1, threads=16)
    per_i = _per_signal_rel(yis, refi)
    assert per_i.max() <= TOL[dtype], (N, int(pick[per_i.argmax()]), per_i.max())
    torch.cuda.empty_cache()
