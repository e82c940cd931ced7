"""Faults everywhere the method protects (Sec. 2.2 fault model and error
propagation; Sec. 5.3 injection protocol), through the C ABI.

A single-bit flip is injected in registers inside the kernel: after any radix
stage of a single-pass transform, in the column pass or the row pass of a
two-pass transform (where the column pass's detection and correction write
the library's workspace), and just above the detection threshold at a group
size where the location code is noisy (the location fallback).  Every
significant flip must be detected, located and corrected: the hit signal
ends within the acceptance tolerance of its fault-free output, every other
signal is bit-identical to the fault-free run.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import abft_model as am
import synth
from groups import group_of

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = {torch.complex64: 2e-6, torch.complex128: 1e-13}
NPDT = {torch.complex64: np.complex64, torch.complex128: np.complex128}
# a flip of a high mantissa bit changes the value by a large fraction of itself
BIG = {torch.complex64: 21, torch.complex128: 50}
TOP = {torch.complex64: 30, torch.complex128: 62}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(xd, dtype, sig, elem, part, bit, pass_, stage):
    y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    tf.inject_arm(sig, elem, part, bit, dtype=dtype, pass_=pass_, stage=stage)
    y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
    torch.cuda.synchronize()
    return y0, y, tf.counts_dict(counts)


def _check_repaired(y0, y, c, sig, dtype, msg):
    assert c["detected"] == 1 and c["uncorrectable"] == 0, msg
    assert c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == sig, msg
    e = oracle.rel_l2(y[sig].cpu().numpy(), y0[sig].cpu().numpy())
    assert e <= TOL[dtype], msg + f" hit signal rel {e:.3e}"
    others = torch.ones(y.shape[0], dtype=torch.bool, device=y.device)
    others[sig] = False
    assert torch.equal(y[others], y0[others]), msg


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 4096), (torch.complex64, 256),
                                     (torch.complex128, 1024)], ids=["fp32-4096", "fp32-256", "fp64-1024"])
def test_flip_after_every_stage_single_pass(dev, dtype, N):
    info = tf.route_info(N, dtype)
    assert info["passes"] == 1
    batch = 40
    x = synth.signals(batch, N, seed=9000 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    rng = np.random.default_rng(N)
    for stage in range(info["stages0"]):
        for bit in (BIG[dtype], TOP[dtype]):
            sig, elem, part = int(rng.integers(0, batch)), int(rng.integers(0, N)), int(rng.integers(0, 2))
            y0, y, c = _run(xd, dtype, sig, elem, part, bit, 0, stage)
            _check_repaired(y0, y, c, sig, dtype, f"N={N} stage={stage} bit={bit} sig={sig} elem={elem} {c}")
    ref = oracle.fft(x[[0, batch - 1]], threads=8)
    assert oracle.rel_l2(y.cpu().numpy()[[0, batch - 1]], ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 1 << 16), (torch.complex64, 1 << 20),
                                     (torch.complex128, 1 << 16)], ids=["fp32-2^16", "fp32-2^20", "fp64-2^16"])
def test_flip_in_column_pass_and_row_pass(dev, dtype, N):
    """A flip in the column pass corrupts the intermediate in the workspace
    unless that pass's own check repairs it; a flip inside the row pass
    (after an intermediate stage) is repaired by the row pass's check."""
    info = tf.route_info(N, dtype)
    assert info["passes"] == 2
    batch = 9
    x = synth.signals(batch, N, seed=9100 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    rng = np.random.default_rng(N + 1)
    cases = [(0, -1), (0, 0), (1, 0), (1, -1)]
    if info["stages0"] > 2:
        cases.append((0, 1))
    for pass_, stage in cases:
        for bit in (BIG[dtype], TOP[dtype]):
            sig, elem, part = int(rng.integers(0, batch)), int(rng.integers(0, N)), int(rng.integers(0, 2))
            y0, y, c = _run(xd, dtype, sig, elem, part, bit, pass_, stage)
            _check_repaired(y0, y, c, sig, dtype,
                            f"N={N} pass={pass_} stage={stage} bit={bit} sig={sig} elem={elem} {c}")
    ref = oracle.fft(x[[sig]], threads=8)
    assert oracle.rel_l2(y.cpu().numpy()[[sig]], ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype,N", [(torch.complex128, 256), (torch.complex64, 512)], ids=["fp64-256", "fp32-512"])
def test_detection_bound_sampled_over_stages_and_positions(dev, dtype, N):
    """GPU counterpart of the brute-force detection check of the reference
    model: a flip far above the threshold after any stage, at any position,
    is always detected and repaired."""
    info = tf.route_info(N, dtype)
    batch = 12
    x = synth.signals(batch, N, seed=9200 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    rng = np.random.default_rng(N + 2)
    for stage in range(info["stages0"]):
        for elem in sorted(set([0, N - 1] + rng.integers(0, N, size=10).tolist())):
            sig, part = int(rng.integers(0, batch)), int(rng.integers(0, 2))
            tf.inject_arm(sig, elem, part, BIG[dtype], dtype=dtype, pass_=0, stage=stage)
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
            c = tf.counts_dict(counts)
            _check_repaired(y0, y, c, sig, dtype, f"stage={stage} elem={elem} sig={sig} {c}")


def test_location_fallback_just_above_threshold(dev):
    """fp64, 1024 points, groups of T = 16 signals: a flip of an output value
    of 1.2-2x the threshold makes the location code D1/D0 noisy; when it is
    not an index the kernel re-encodes the group's signals one by one and
    corrects the one whose checksums disagree (counts.fallback).  Every
    detected flip is corrected and every signal ends within the tolerance of
    its fault-free output."""
    dtype, N, T = torch.complex128, 1024, 16
    old = tf.get_tuning(N, dtype)
    old_gran = tf.route_info(N, dtype)["gran"]
    tf.set_tuning(N, dtype, T=T)
    tf.set_granularity(N, dtype, 0)   # the location code belongs to the per-group check
    try:
        info = tf.route_info(N, dtype)
        assert info["gran"] == 0 and info["T"] == T, info
        kappa = tf.get_tuning(N, dtype)[1]
        batch = 4 * T
        x = synth.signals(batch, N, seed=9300, dtype=np.complex128)
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        yc = y0.cpu().numpy()
        u = 2.0 ** -53
        rng = np.random.default_rng(9301)
        fallbacks = detected = 0
        for trial in range(40):
            sig, elem, part = int(rng.integers(0, batch)), int(rng.integers(0, N)), int(rng.integers(0, 2))
            members = group_of(sig, batch, info)
            assert sig in members and len(members) == T
            nu = float(np.sum(np.abs(x[members]) ** 2))
            tau = kappa * u * math.sqrt(N * math.log2(N)) * math.sqrt(nu)
            v = yc[sig, elem].real if part == 0 else yc[sig, elem].imag
            if v == 0.0:
                continue
            # a mantissa bit j of v moves it by 2^(exponent(v) + j - 52)
            e = math.frexp(abs(v))[1] - 1
            target = float(rng.uniform(1.2, 2.0)) * tau
            bit = int(round(math.log2(target) - e + 52))
            if not (0 <= bit <= 51):
                continue
            tf.inject_arm(sig, elem, part, bit, dtype=dtype)
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
            c = tf.counts_dict(counts)
            msg = f"trial={trial} sig={sig} elem={elem} bit={bit} {c}"
            # near the threshold the location code may name a neighbour; the
            # threshold keeps every signal within the tolerance either way
            yh = y.cpu().numpy()
            err = np.linalg.norm(yh - yc, axis=1) / np.linalg.norm(yc, axis=1)
            assert err.max() <= TOL[dtype], msg + f" rel {err.max():.3e} at {err.argmax()}"
            if c["detected"]:
                detected += 1
                assert c["uncorrectable"] == 0 and c["corrected"] + c["rebuilt"] == 1, msg
                fallbacks += c["fallback"]
            if fallbacks >= 3:
                break
        print(f"fallback: {fallbacks} of {detected} detected flips just above the threshold")
        assert fallbacks >= 1, (fallbacks, detected)
    finally:
        tf.set_tuning(N, dtype, T=old[0], kappa=old[1])
        tf.set_granularity(N, dtype, old_gran)


@pytest.mark.parametrize("mode", ["persistent", "per_size"])
def test_ragged_flip_in_column_pass(dev, mode):
    sizes = [1 << 14] * 4 + [3 << 13] * 3 + [512] * 10
    total = int(sum(sizes))
    x_host = synth.signals(1, total, seed=9400, dtype=np.complex64).reshape(-1)
    x = torch.from_numpy(x_host).to(dev)
    plan = tf.RaggedPlan(sizes, device=dev)
    y0, _ = plan(x, ft_mode=tf.FT_OFF, mode=mode)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for sig, pass_, stage in [(1, 0, -1), (5, 0, 0), (2, 1, 0), (12, 0, 1)]:
        counts = tf.new_counts(dev)
        tf.inject_arm(sig, sizes[sig] // 3, 1, BIG[torch.complex64], dtype=torch.complex64,
                      pass_=pass_, stage=stage)
        y, _ = plan(x, ft_mode=tf.FT_CORRECT, counts=counts, mode=mode)
        torch.cuda.synchronize()
        c = tf.counts_dict(counts)
        msg = f"{mode} sig={sig} pass={pass_} stage={stage} {c}"
        assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == sig, msg
        a, b = int(off[sig]), int(off[sig + 1])
        assert oracle.rel_l2(y[a:b].cpu().numpy(), y0[a:b].cpu().numpy()) <= TOL[torch.complex64], msg
        keep = torch.ones(total, dtype=torch.bool, device=dev)
        keep[a:b] = False
        assert torch.equal(y[keep], y0[keep]), msg
    plan.close()
