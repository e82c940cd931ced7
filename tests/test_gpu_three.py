"""Three-pass transforms through the C ABI (Sec. 3.3: three launches for
lengths 2^23..2^29; Sec. 3.1 multi-pass decomposition N = N1 N2 N3).

Pass 0 is a column pass of N1 over the M = N2 N3 columns, pass 1 a column
pass of N2 within each row of M with the outer twiddle at its load, pass 2 a
row pass of N3 whose store transposes to the output order.  Each pass runs
its own two-side checksums (Sec. 4).  Checked against the CPU fp64 oracle:
relative L2 <= 2e-6 per signal in fp32 at 2^23 and 2^24 (default routes),
at 2^22 on a forced three-pass route (against the oracle and the two-pass
route), every built three-pass route of 2^23 over chunks with a ragged last
one, the inverse, in place, ABFT on / off bit identity, and a bit flip in
each pass and at several stages detected, reported against the caller's
signal and repaired.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

DT = torch.complex64
TOL = 2e-6
BIG, TOP = 21, 30


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _per_signal_rel(got, ref):
    num = np.linalg.norm(got - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    return num / np.maximum(den, 1e-300)


def _restore(N):
    tf.set_route(N, DT, 0)
    tf.set_chunk(N, DT, 128 << 20)
    import os
    if os.path.exists(tf._lib.TUNING_PATH):
        tf.load_tuning(tf._lib.TUNING_PATH)


@pytest.mark.parametrize("N", [1 << 23, 1 << 24], ids=["2^23", "2^24"])
def test_default_route_parity_and_ft_identity(dev, N):
    info = tf.route_info(N, DT)
    assert info["passes"] == 3 and info["N1"] * info["N2"] * info["N3"] == N, info
    # 2^23: two signals per 128 MiB chunk, so batch 3 ends on a ragged chunk
    batch = 3 if N == 1 << 23 else 2
    x = synth.signals(batch, N, seed=7300 + N.bit_length())
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, threads=8)
    y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    y0h = y0.cpu().numpy()
    rel = _per_signal_rel(y0h, ref)
    assert rel.max() <= TOL, rel
    for ft in (tf.FT_DETECT, tf.FT_CORRECT):
        y, counts = tf.fft_c2c(xd, ft_mode=ft)
        c = tf.counts_dict(counts)
        assert c["detected"] == 0, (ft, c)
        assert torch.equal(y, y0), ft
    # inverse of the forward output, scaled 1/N, returns the input
    xi, counts = tf.fft_c2c(y0, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT)
    assert tf.counts_dict(counts)["detected"] == 0
    refi = oracle.fft(y0h, dir=1, threads=8)
    assert _per_signal_rel(xi.cpu().numpy(), refi).max() <= TOL


def test_forced_three_pass_at_2_22_matches_two_pass_and_oracle(dev):
    N = 1 << 22
    codes = [c for c in tf.routes(N, DT) if tf.route_n2(c)]
    assert codes, "no three-pass route of 2^22"
    batch = 3
    x = synth.signals(batch, N, seed=7322)
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, threads=8)
    try:
        y2, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)   # the two-pass default
        assert tf.route_info(N, DT)["passes"] == 2
        for code in codes:
            tf.set_route(N, DT, code)
            assert tf.get_route(N, DT) == code
            info = tf.route_info(N, DT)
            assert info["passes"] == 3 and info["N2"] == tf.route_n2(code), info
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
            assert tf.counts_dict(counts)["detected"] == 0, hex(code)
            rel = _per_signal_rel(y.cpu().numpy(), ref)
            assert rel.max() <= TOL, (hex(code), rel)
            # both decompositions meet the oracle; they need not agree bitwise
            assert oracle.rel_l2(y.cpu().numpy(), y2.cpu().numpy()) <= 2 * TOL
    finally:
        _restore(N)


def test_every_three_pass_route_of_2_23_over_chunks(dev):
    N = 1 << 23
    codes = [c for c in tf.routes(N, DT) if tf.route_n2(c)]
    assert len(codes) >= 2, codes
    batch = 3
    x = synth.signals(batch, N, seed=7323)
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, threads=8)
    try:
        # one signal per chunk: three chunks
        tf.set_chunk(N, DT, N * 8)
        for code in codes:
            tf.set_route(N, DT, code)
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
            assert tf.counts_dict(counts)["detected"] == 0, hex(code)
            rel = _per_signal_rel(y.cpu().numpy(), ref)
            assert rel.max() <= TOL, (hex(code), rel)
    finally:
        _restore(N)


def test_in_place(dev):
    N = 1 << 23
    batch = 2
    x = synth.signals(batch, N, seed=7330)
    ref = oracle.fft(x, threads=8)
    xd = torch.from_numpy(x).to(dev)
    y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT, out=xd)
    assert y.data_ptr() == xd.data_ptr()
    assert tf.counts_dict(counts)["detected"] == 0
    assert _per_signal_rel(xd.cpu().numpy(), ref).max() <= TOL


@pytest.mark.parametrize("N,forced", [(1 << 22, True), (1 << 23, False)], ids=["2^22-forced", "2^23"])
def test_flip_in_each_pass_is_repaired(dev, N, forced):
    """A flip in pass 0 or 1 would spread through the later passes over the
    whole signal unless that pass's own check repairs it before its store;
    a flip in pass 2 reaches the output directly."""
    try:
        if forced:
            tf.set_route(N, DT, [c for c in tf.routes(N, DT) if tf.route_n2(c)][0])
        info = tf.route_info(N, DT)
        assert info["passes"] == 3
        batch = 3
        x = synth.signals(batch, N, seed=7400 + N.bit_length())
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        rng = np.random.default_rng(N + 5)
        stages = (info["stages0"], info["stages1"], info["stages2"])
        for pass_ in (0, 1, 2):
            for stage in sorted({0, -1, stages[pass_] - 2}):
                for bit in (BIG, TOP):
                    sig, elem, part = int(rng.integers(0, batch)), int(rng.integers(0, N)), int(rng.integers(0, 2))
                    msg = f"N={N} pass={pass_} stage={stage} bit={bit} sig={sig} elem={elem}"
                    tf.inject_arm(sig, elem, part, bit, dtype=DT, pass_=pass_, stage=stage)
                    y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
                    c = tf.counts_dict(counts)
                    assert c["detected"] == 1 and c["uncorrectable"] == 0, (msg, c)
                    assert c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == sig, (msg, c)
                    e = oracle.rel_l2(y[sig].cpu().numpy(), y0[sig].cpu().numpy())
                    assert e <= TOL, (msg, e)
                    others = torch.ones(batch, dtype=torch.bool, device=dev)
                    others[sig] = False
                    assert torch.equal(y[others], y0[others]), msg
        ref = oracle.fft(x[[sig]], threads=8)
        assert oracle.rel_l2(y.cpu().numpy()[[sig]], ref) <= TOL
    finally:
        _restore(N)


def test_flip_detected_without_correction(dev):
    N = 1 << 23
    batch = 2
    x = synth.signals(batch, N, seed=7450)
    xd = torch.from_numpy(x).to(dev)
    for pass_ in (0, 1, 2):
        tf.inject_arm(1, 12345 + pass_, 0, TOP, dtype=DT, pass_=pass_, stage=-1)
        _, counts = tf.fft_c2c(xd, ft_mode=tf.FT_DETECT)
        c = tf.counts_dict(counts)
        assert c["detected"] >= 1 and c["corrected"] == 0 and c["last_signal"] == 1, (pass_, c)


def test_noalloc_rejects_three_pass(dev):
    """Two intermediates of one signal exceed the no-allocation scratch."""
    N = 1 << 23
    xd = torch.zeros(1, N, dtype=DT, device=dev)
    out = torch.empty_like(xd)
    with pytest.raises(RuntimeError):
        tf.fft_c2c_noalloc(xd, out, ft_mode=tf.FT_OFF)


def test_capture_after_prepare(dev):
    """tfft_prepare reserves the two intermediates of a three-pass chunk, so
    a captured call allocates nothing; replays with new data match the eager
    result bit for bit (eager work between replays)."""
    N, batch = 1 << 23, 2
    s = torch.cuda.Stream(device=dev)
    x = torch.empty(batch, N, dtype=DT, device=dev)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    with torch.cuda.stream(s):
        tf.prepare(N, DT, tf.FT_CORRECT, batch=batch)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tf.fft_c2c(x, ft_mode=tf.FT_CORRECT, out=y, counts=counts)
    torch.cuda.synchronize()
    for r in range(3):
        fresh = synth.signals(batch, N, seed=7500 + r)
        x.copy_(torch.from_numpy(fresh).to(dev))
        with torch.cuda.stream(s):
            eager, _ = tf.fft_c2c(x, ft_mode=tf.FT_CORRECT)
        torch.cuda.synchronize()
        counts.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), r
        assert tf.counts_dict(counts)["detected"] == 0
    ref = oracle.fft(fresh[[1]], threads=8)
    assert _per_signal_rel(y.cpu().numpy()[[1]], ref).max() <= TOL


def test_offline_abft_on_three_pass_length(dev):
    """The unfused baseline runs on the three-pass transform too: clean
    output equals the fused path's plain output; a flip in the last pass is
    detected and the signal rebuilt."""
    N, batch = 1 << 23, 2
    x = synth.signals(batch, N, seed=7550)
    xd = torch.from_numpy(x).to(dev)
    y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    y, counts = tf.fft_c2c_offline(xd)
    assert tf.counts_dict(counts)["detected"] == 0
    assert torch.equal(y, y0)
    tf.inject_arm(1, 4321, 0, 30, dtype=DT, pass_=2)
    y, counts = tf.fft_c2c_offline(xd)
    c = tf.counts_dict(counts)
    assert c["detected"] == 1 and c["rebuilt"] == 1 and c["last_signal"] == 1, c
    assert oracle.rel_l2(y[1].cpu().numpy(), y0[1].cpu().numpy()) <= TOL
    assert torch.equal(y[0], y0[0])
