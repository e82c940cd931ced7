"""Thread-level two-side ABFT (Sec. 4.2): every radix-R DFT in registers is
checked, located and corrected on its own, through the C ABI
(TFFT_FT_THREAD).  Fault-free: no detection, outputs bit-identical to the
plain kernel of the same plan and within the oracle tolerance.  A bit flip
injected between a DFT and its check, at any stage: detected, located,
corrected; the hit signal ends within the tolerance of its fault-free
output and every other signal is bit-identical."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = {torch.complex64: 2e-6, torch.complex128: 1e-13}
NPDT = {torch.complex64: np.complex64, torch.complex128: np.complex128}
BITS = {torch.complex64: (21, 26, 30), torch.complex128: (50, 56, 62)}
CASES = [(torch.complex64, 256), (torch.complex64, 1024), (torch.complex64, 4096), (torch.complex64, 8192),
         (torch.complex128, 512), (torch.complex128, 2048)]
IDS = [f"{'fp32' if d == torch.complex64 else 'fp64'}-{n}" for d, n in CASES]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rel(got, ref):
    return np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


@pytest.mark.parametrize("dtype,N", CASES, ids=IDS)
def test_clean_matches_plain_and_oracle(dev, dtype, N):
    batch = max(8, (1 << 18) // N) + 3
    x = synth.signals(batch, N, seed=9500 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    tf.set_route(N, dtype, tf.get_route(N, dtype, tf.FT_CORRECT))
    try:
        y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_THREAD)
        c = tf.counts_dict(counts)
        assert c["detected"] == 0, c
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        assert torch.equal(y, y0)
        ref = oracle.fft(x[[0, batch // 2, batch - 1]], threads=8)
        assert _rel(y.cpu().numpy()[[0, batch // 2, batch - 1]], ref).max() <= TOL[dtype]
        yi, counts = tf.fft_c2c(xd, dir=tf.INVERSE, ft_mode=tf.FT_THREAD)
        assert tf.counts_dict(counts)["detected"] == 0
        refi = oracle.fft(x[[1]], dir=1, threads=8)
        assert _rel(yi.cpu().numpy()[[1]], refi).max() <= TOL[dtype]
    finally:
        tf.set_route(N, dtype, 0)
        import os
        if os.path.exists(tf._lib.TUNING_PATH):
            tf.load_tuning(tf._lib.TUNING_PATH)


@pytest.mark.parametrize("dtype,N", CASES, ids=IDS)
def test_flip_in_any_stage_is_corrected(dev, dtype, N):
    batch = 24
    x = synth.signals(batch, N, seed=9600 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    info = tf.route_info(N, dtype, tf.FT_CORRECT)
    assert info["passes"] == 1
    y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    rng = np.random.default_rng(N)
    for stage in range(info["stages0"]):
        for bit in BITS[dtype]:
            sig, elem, part = int(rng.integers(0, batch)), int(rng.integers(0, N)), int(rng.integers(0, 2))
            msg = f"N={N} stage={stage} bit={bit} sig={sig} elem={elem}"
            tf.inject_arm(sig, elem, part, bit, dtype=dtype, pass_=0, stage=stage)
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_THREAD)
            c = tf.counts_dict(counts)
            assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1 and c["uncorrectable"] == 0, (msg, c)
            assert c["last_signal"] == sig, (msg, c)
            assert _rel(y[sig].cpu().numpy(), y0[sig].cpu().numpy()) <= TOL[dtype], msg
            others = torch.ones(batch, dtype=torch.bool, device=dev)
            others[sig] = False
            assert torch.equal(y[others], y0[others]), msg


def test_no_false_alarm_at_scale(dev):
    """2^24 elements of fp32 at 4096 points: some 10^7 checked DFTs."""
    N = 4096
    g = torch.Generator(device=dev)
    g.manual_seed(9700)
    x = (torch.rand(1 << 24, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(-1, N)
    for d in (tf.FORWARD, tf.INVERSE):
        _, counts = tf.fft_c2c(x, dir=d, ft_mode=tf.FT_THREAD)
        assert tf.counts_dict(counts)["detected"] == 0, d


def test_two_pass_lengths_unsupported(dev):
    xd = torch.zeros(2, 1 << 16, dtype=torch.complex64, device=dev)
    with pytest.raises(RuntimeError):
        tf.fft_c2c(xd, ft_mode=tf.FT_THREAD)
