"""Offline (unfused) two-side ABFT (tfft_c2c_offline), the baseline the fused
kernels are compared with (Sec. 2.2 offline FT-FFT, Sec. 5.2).

Its transform is the plain kernel's, so without a fault the output equals
tfft_c2c with ABFT off bit for bit (and the oracle within tolerance) and
nothing is counted; a flip in the plain transform is detected by the
separate checksum passes and the signal rebuilt from the right-side sums of
its group of 16 (Eq. 5); two faults in one group are counted uncorrectable.
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


CASES = [(torch.complex64, 256, 40), (torch.complex64, 4096, 37), (torch.complex64, 1 << 16, 19),
         (torch.complex128, 1024, 33), (torch.complex128, 1 << 16, 17)]
IDS = ["fp32-256", "fp32-4096", "fp32-2^16", "fp64-1024", "fp64-2^16"]


@pytest.mark.parametrize("dtype,N,batch", CASES, ids=IDS)
@pytest.mark.parametrize("dir", [-1, 1], ids=["fwd", "inv"])
def test_offline_matches_plain_and_oracle(dev, dtype, N, batch, dir):
    x = synth.signals(batch, N, seed=9900 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    y0, _ = tf.fft_c2c(xd, dir=dir, ft_mode=tf.FT_OFF)
    y, c = tf.fft_c2c_offline(xd, dir=dir)
    torch.cuda.synchronize()
    cd = tf.counts_dict(c)
    assert cd["detected"] == 0 and cd["uncorrectable"] == 0, cd
    assert torch.equal(y, y0)
    pick = [0, batch // 2, batch - 1]
    ref = oracle.fft(x[pick], dir=dir, threads=8)
    assert oracle.rel_l2(y.cpu().numpy()[pick], ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype,N,batch", CASES, ids=IDS)
def test_offline_detects_and_rebuilds(dev, dtype, N, batch):
    x = synth.signals(batch, N, seed=9950 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    yc = y0.cpu().numpy()
    bit = 29 if dtype == torch.complex64 else 61
    for sig, stage in ((batch - 1, -1), (batch // 3, 0)):
        tf.inject_arm(sig, N // 5, 1, bit, dtype=dtype, stage=stage)
        y, c = tf.fft_c2c_offline(xd)
        cd = tf.counts_dict(c)
        msg = f"N={N} sig={sig} stage={stage} {cd}"
        assert cd["detected"] == 1 and cd["rebuilt"] == 1 and cd["last_signal"] == sig, msg
        yh = y.cpu().numpy()
        assert oracle.rel_l2(yh[sig], yc[sig]) <= TOL[dtype], msg
        keep = np.ones(batch, bool)
        keep[sig] = False
        assert np.array_equal(yh[keep], yc[keep]), msg
    # two faults in one group of 16 consecutive signals
    tf.inject_arm(1, 3, 0, bit, dtype=dtype, signal2=2)
    y, c = tf.fft_c2c_offline(xd)
    cd = tf.counts_dict(c)
    assert cd["detected"] == 2 and cd["uncorrectable"] == 2 and cd["rebuilt"] == 0, cd


def test_offline_in_place_and_inverse_round_trip(dev):
    N, batch = 2048, 20
    x = synth.signals(batch, N, seed=9990)
    xd = torch.from_numpy(x).to(dev)
    y, c = tf.fft_c2c_offline(xd.clone(), out=None)
    z = y.clone()
    z2, c2 = tf.fft_c2c_offline(z, dir=1, out=z)   # in place
    assert tf.counts_dict(c)["detected"] == 0 and tf.counts_dict(c2)["detected"] == 0
    assert oracle.rel_l2(z2.cpu().numpy(), x) <= 2e-6


@pytest.mark.parametrize("N,batch", [(1 << 20, 128), (1 << 22, 32)], ids=["2^20", "2^22"])
def test_offline_no_false_alarm_at_large_N(dev, N, batch):
    """The offline checksums of long signals are sums over millions of
    elements added by many workgroups in no fixed order; kept in double they
    stay far below the threshold (fp32 totals raised false alarms here)."""
    g = torch.Generator(device=dev)
    g.manual_seed(9995 + N)
    x = (torch.rand(batch, N, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(batch, N)
    for _ in range(3):
        y, c = tf.fft_c2c_offline(x)
        cd = tf.counts_dict(c)
        assert cd["detected"] == 0, cd
    y0, _ = tf.fft_c2c(x, ft_mode=tf.FT_OFF)
    assert torch.equal(y, y0)
