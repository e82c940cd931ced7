"""Gradient of L = sum(w * |FFT(x)|^2) through the hand-written adjoint.

Checked against the oracle gradient 2 * (unscaled inverse DFT)(w * y) (pinned
on the CPU by finite differences and by torch.autograd on torch.fft), and by
central finite differences of the GPU loss itself in fp64.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import abft_model as am
import synth

pytestmark = pytest.mark.gpu
tf = pytest.importorskip("paper_2412_05824_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _loss(xd, wd, ft=2, counts=None):
    y = tf.FFT.apply(xd, ft, counts)
    return (wd * (y.real ** 2 + y.imag ** 2)).sum()


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 2e-6), (torch.complex128, 1e-13)],
                         ids=["fp32", "fp64"])
@pytest.mark.parametrize("N", [256, 4096, 1 << 14])
def test_gradient_matches_oracle(dev, dtype, tol, N):
    rows = max(4, (1 << 17) // N)
    npdt = np.complex64 if dtype == torch.complex64 else np.complex128
    rdt = np.float32 if dtype == torch.complex64 else np.float64
    x = synth.signals(rows, N, seed=7000 + N, dtype=npdt)
    w = synth.weights((rows, N), seed=7100 + N, dtype=rdt)
    xd = torch.from_numpy(x).to(dev).requires_grad_(True)
    wd = torch.from_numpy(w).to(dev)
    counts = tf.new_counts(dev)
    loss = _loss(xd, wd, counts=counts)
    loss.backward()
    g = xd.grad.detach().cpu().numpy()
    ref = am.grad_sum_w_abs2(x.astype(np.complex128), w.astype(np.float64))
    assert oracle.rel_l2(g, ref) <= tol, N
    c = tf.counts_dict(counts)
    assert c["detected"] == 0, c


def test_gradient_finite_differences_fp64(dev):
    # central differences of the GPU loss itself, fp64, h = 1e-6, [4, 64] slice
    rows, N = 4, 1024
    x = synth.signals(rows, N, seed=11, dtype=np.complex128)
    w = synth.weights((rows, N), seed=12, dtype=np.float64)
    xd = torch.from_numpy(x).to(dev).requires_grad_(True)
    wd = torch.from_numpy(w).to(dev)
    _loss(xd, wd).backward()
    g = xd.grad.detach().cpu().numpy()
    h = 1e-6
    fd = np.zeros((rows, 64), complex)
    with torch.no_grad():
        base = xd.detach().clone()
        for r in range(rows):
            for n in range(64):
                vals = []
                for d in (h, -h, 1j * h, -1j * h):
                    xp = base.clone()
                    xp[r, n] += d
                    vals.append(float(_loss(xp, wd)))
                fd[r, n] = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
    # FD noise: u * |L| / h ~ 1e-16 * 1e6 / 1e-6 = 1e-4 against gradients ~ 1e3
    assert oracle.rel_l2(g[:, :64], fd) < 1e-6


def test_gradient_with_injected_fault_in_backward(dev):
    # a bit flip inside the adjoint transform is corrected like any other
    rows, N = 64, 2048
    x = synth.signals(rows, N, seed=21, dtype=np.complex64)
    w = synth.weights((rows, N), seed=22, dtype=np.float32)
    xd = torch.from_numpy(x).to(dev).requires_grad_(True)
    wd = torch.from_numpy(w).to(dev)
    counts = tf.new_counts(dev)
    loss = _loss(xd, wd, counts=counts)
    tf.inject_arm(17, 99, 0, 29, dtype=torch.complex64)   # armed for the backward call
    loss.backward()
    c = tf.counts_dict(counts)
    assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == 17, c
    ref = am.grad_sum_w_abs2(x.astype(np.complex128), w.astype(np.float64))
    assert oracle.rel_l2(xd.grad.detach().cpu().numpy(), ref) <= 2e-6
