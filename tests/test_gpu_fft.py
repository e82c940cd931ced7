"""GPU parity: the HIP path through the C ABI against the CPU fp64 oracle.

Transform (Sec. 2.2): relative L2 <= 2e-6 (fp32), <= 1e-13 (fp64) per batch
and per signal.  Fault tolerance (Sec. 4): with no fault the ABFT kernels
produce bit-identical outputs to the plain kernels and count nothing; an
injected bit flip (Sec. 5.3 protocol) that exceeds the threshold is detected,
located and corrected back within the same tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import abft_model as am
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = {torch.complex64: 2e-6, torch.complex128: 1e-13}
NPDT = {torch.complex64: np.complex64, torch.complex128: np.complex128}
PREC = {torch.complex64: "fp32", torch.complex128: "fp64"}
SIZES = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
# lengths served by a column pass and a row pass (N = N1 * N2)
TWO_PASS = {torch.complex64: [1 << 14, 1 << 15, 1 << 17, 1 << 20],
            torch.complex128: [1 << 13, 1 << 14, 1 << 16]}
DTYPES = [torch.complex64, torch.complex128]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _batch_for(N):
    # several workgroups plus a ragged tail that fills no whole group
    return max(3, (1 << 17) // N) + 3


def _per_signal_rel(got, ref):
    num = np.linalg.norm(got - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    return num / np.maximum(den, 1e-300)


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
@pytest.mark.parametrize("N", SIZES)
def test_forward_parity_and_ft_bit_identity(dev, N, dtype):
    batch = _batch_for(N)
    x = synth.signals(batch, N, seed=2000 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, threads=8)
    # the modes agree bit for bit on one plan; the tuning table may give each
    # mode its own, so pin the correcting mode's while comparing
    tf.set_route(N, dtype, tf.get_route(N, dtype, tf.FT_CORRECT))
    try:
        y0, _ = tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=tf.FT_OFF)
        y0h = y0.cpu().numpy()
        assert oracle.rel_l2(y0h, ref) <= TOL[dtype]
        assert _per_signal_rel(y0h, ref).max() <= TOL[dtype]
        for ft in (tf.FT_DETECT, tf.FT_CORRECT):
            y, counts = tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=ft)
            c = tf.counts_dict(counts)
            assert c["detected"] == 0, (ft, c)
            # ABFT must not touch the data path
            assert torch.equal(y, y0), ft
    finally:
        tf.set_route(N, dtype, 0)
        _restore_tuning()
    # and each mode's own tuned plan matches the oracle
    for ft in (tf.FT_OFF, tf.FT_CORRECT):
        y, _ = tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=ft)
        assert _per_signal_rel(y.cpu().numpy(), ref).max() <= TOL[dtype], ft


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
@pytest.mark.parametrize("N", [64, 512, 2048, 4096])
def test_inverse_parity_and_round_trip(dev, N, dtype):
    batch = _batch_for(N) // 2 + 1
    x = synth.signals(batch, N, seed=3000 + N, dist="normal", dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, dir=+1, threads=8)
    for ft in (tf.FT_OFF, tf.FT_CORRECT):
        y, counts = tf.fft_c2c(xd, dir=tf.INVERSE, ft_mode=ft)
        assert oracle.rel_l2(y.cpu().numpy(), ref) <= TOL[dtype]
        if counts is not None:
            assert tf.counts_dict(counts)["detected"] == 0
    yf, _ = tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=tf.FT_CORRECT)
    xr, _ = tf.fft_c2c(yf, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT)
    # a round trip is two transforms: their errors add
    assert oracle.rel_l2(xr.cpu().numpy(), x) <= 2 * TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
def test_in_place_and_explicit_scale(dev, dtype):
    N, batch = 1024, 37
    x = synth.signals(batch, N, seed=77, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=tf.FT_CORRECT, out=xd)
    assert oracle.rel_l2(xd.cpu().numpy(), oracle.fft(x)) <= TOL[dtype]
    xd2 = torch.from_numpy(x).to(dev)
    y, _ = tf.fft_c2c(xd2, dir=tf.FORWARD, ft_mode=tf.FT_OFF, scale=0.5)
    assert oracle.rel_l2(y.cpu().numpy(), 0.5 * oracle.fft(x)) <= TOL[dtype]


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 8192), (torch.complex64, 16384),
                                     (torch.complex128, 2048), (torch.complex128, 4096),
                                     (torch.complex128, 8192)],
                         ids=["fp32-8192", "fp32-16384", "fp64-2048", "fp64-4096", "fp64-8192"])
def test_in_place_correction_on_table_encoded_single_passes(dev, dtype, N):
    """In place, the correcting kernels keep the group's input sums in
    registers (the inputs are overwritten); these lengths encode with the
    cotangent form of e^T W read from the table.  Clean: equal to the
    out-of-place output, within tolerance of the oracle; one exponent flip:
    detected, the signal repaired to the clean output's tolerance, the others
    untouched."""
    batch = _batch_for(N)
    x = synth.signals(batch, N, seed=2600 + N, dtype=NPDT[dtype])
    ref = oracle.fft(x, threads=8)
    y0, _ = tf.fft_c2c(torch.from_numpy(x).to(dev), ft_mode=tf.FT_CORRECT)
    xd = torch.from_numpy(x).to(dev)
    y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT, out=xd)
    assert y.data_ptr() == xd.data_ptr()
    assert tf.counts_dict(counts)["detected"] == 0
    assert torch.equal(xd, y0)
    assert _per_signal_rel(xd.cpu().numpy(), ref).max() <= TOL[dtype]
    sig, elem = batch // 2, N // 3
    bit = 28 if dtype == torch.complex64 else 60
    xd = torch.from_numpy(x).to(dev)
    tf.inject_arm(sig, elem, 0, bit, dtype=dtype)
    y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT, out=xd)
    c = tf.counts_dict(counts)
    assert c["detected"] == 1 and c["uncorrectable"] == 0 and c["last_signal"] == sig, c
    assert c["corrected"] + c["rebuilt"] == 1, c
    yh, y0h = xd.cpu().numpy(), y0.cpu().numpy()
    assert oracle.rel_l2(yh[sig], y0h[sig]) <= TOL[dtype]
    others = np.ones(batch, bool)
    others[sig] = False
    assert np.array_equal(yh[others], y0h[others])


def test_empty_batch_and_single_signal(dev):
    x = torch.zeros(0, 256, dtype=torch.complex64, device=dev)
    y, _ = tf.fft_c2c(x, ft_mode=tf.FT_OFF)
    assert y.shape == (0, 256)
    x1 = synth.signals(1, 256, seed=5, dtype=np.complex64)
    y1, c = tf.fft_c2c(torch.from_numpy(x1).to(dev), ft_mode=tf.FT_CORRECT)
    assert oracle.rel_l2(y1.cpu().numpy(), oracle.fft(x1)) <= 2e-6
    assert tf.counts_dict(c)["detected"] == 0


def _inject_case(dev, dtype, N, batch, sig, elem, part, bit, T=None):
    x = synth.signals(batch, N, seed=4000 + N, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    ref = oracle.fft(x, threads=8)
    y_clean, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
    yc = y_clean.cpu().numpy()
    tf.inject_arm(sig, elem, part, bit, dtype=dtype)
    y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
    c = tf.counts_dict(counts)
    yh = y.cpu().numpy()
    # the flip the kernel applied, as the model sees it
    flipped = am.flip_bit(complex(yc[sig, elem]), part, bit, PREC[dtype])
    delta = abs(flipped - yc[sig, elem])
    return x, ref, yc, yh, c, delta


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
@pytest.mark.parametrize("N", [64, 256, 1024, 4096])
def test_injected_flip_detected_located_corrected(dev, N, dtype):
    batch = _batch_for(N)
    nbits = 31 if dtype == torch.complex64 else 63
    tol = TOL[dtype]
    rng = np.random.default_rng(N)
    for bit in sorted(set([nbits - 1, nbits - 3, nbits - 8, nbits - 12, nbits // 2, 5, 0] +
                          rng.integers(0, nbits, size=3).tolist())):
        sig = int(rng.integers(0, batch))
        elem = int(rng.integers(0, N))
        part = int(rng.integers(0, 2))
        x, ref, yc, yh, c, delta = _inject_case(dev, dtype, N, batch, sig, elem, part, bit)
        per = _per_signal_rel(yh, ref)
        msg = f"N={N} bit={bit} sig={sig} elem={elem} part={part} delta={delta:.3e} counts={c}"
        # every output, corrupted or not, ends within tolerance of the oracle,
        # and the hit signal within tolerance of its fault-free output
        assert per.max() <= tol, msg + f" worst={per.max():.3e} at {per.argmax()}"
        assert oracle.rel_l2(yh[sig], yc[sig]) <= tol, msg
        if c["detected"]:
            assert c["detected"] == 1 and c["uncorrectable"] == 0, msg
            assert c["corrected"] + c["rebuilt"] == 1, msg
            assert c["last_signal"] == sig, msg
        else:
            # only flips far below the signal's norm may pass unnoticed
            assert delta <= tol * np.linalg.norm(ref[sig]), msg
        # the uncorrupted signals are bit-identical to the clean run
        others = np.ones(batch, bool)
        others[sig] = False
        assert np.array_equal(yh[others], yc[others]), msg


@pytest.mark.parametrize("dtype,N,variant", [(torch.complex64, 8192, 0), (torch.complex64, 2048, 1),
                                             (torch.complex128, 4096, 0)], ids=["fp32-8192", "fp32-2048e8", "fp64-4096"])
def test_resident_loop_late_group(dev, dtype, N, variant):
    """Single-pass checking kernels with one signal per workgroup stay
    resident and loop over the groups; a batch several times the resident
    workgroups, with a flip in a group of a late iteration, must be detected,
    located and corrected like any other, and every other signal must match
    the plain kernel bit for bit."""
    batch = 2600
    elem, part = N // 3, 0
    bit = 30 if dtype == torch.complex64 else 62
    tf.set_route(N, dtype, tf.route_code(1, variant, 0))
    # one transaction per group: 2600 groups, several rounds of the resident
    # workgroups (each group g is signal g); the flip is in the last round
    tf.set_tuning(N, dtype, T=1)
    sig = batch - 7
    try:
        x = synth.signals(batch, N, seed=4100 + N, dtype=NPDT[dtype])
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        y2, c2 = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        assert tf.counts_dict(c2)["detected"] == 0
        assert torch.equal(y2, y0)
        tf.inject_arm(sig, elem, part, bit, dtype=dtype)
        y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        c = tf.counts_dict(counts)
        assert c["detected"] == 1 and c["uncorrectable"] == 0, c
        assert c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == sig, c
        pick = [0, 1, batch // 2, sig, batch - 1]
        ref = oracle.fft(x[pick], threads=8)
        got = y.cpu().numpy()
        for i, s in enumerate(pick):
            assert oracle.rel_l2(got[s], ref[i]) <= TOL[dtype], (N, s)
        assert oracle.rel_l2(got[sig], y0[sig].cpu().numpy()) <= TOL[dtype]
        others = torch.ones(batch, dtype=torch.bool, device=dev)
        others[sig] = False
        assert torch.equal(y[others], y0[others])
    finally:
        tf.set_route(N, dtype, 0)
        _restore_tuning()


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
def test_exponent_flips_always_detected(dev, dtype):
    # the top exponent bits change a value by orders of magnitude (or make it
    # Inf/NaN); they must all be detected and repaired
    N = 512
    batch = _batch_for(N)
    top = [30, 29, 28, 27, 26, 25, 24, 23] if dtype == torch.complex64 else [62, 61, 60, 59, 56, 53, 52]
    for i, bit in enumerate(top):
        sig, elem, part = (7 * i + 3) % batch, (37 * i + 1) % N, i % 2
        x, ref, yc, yh, c, delta = _inject_case(dev, dtype, N, batch, sig, elem, part, bit)
        msg = f"bit={bit} sig={sig} elem={elem} counts={c} delta={delta}"
        assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1, msg
        assert c["last_signal"] == sig, msg
        assert oracle.rel_l2(yh[sig], ref[sig]) <= TOL[dtype], msg
        assert oracle.rel_l2(yh[sig], yc[sig]) <= TOL[dtype], msg


@pytest.mark.parametrize("T", [1, 2, 8])
def test_transactions_per_slot(dev, T):
    # T changes only the grouping of the checksums, never the transform
    N, dtype = 1024, torch.complex64
    old = tf.get_tuning(N, dtype)
    try:
        tf.set_tuning(N, dtype, T=T)
        batch = 3 * T * 4 + 1
        x = synth.signals(batch, N, seed=55, dtype=np.complex64)
        xd = torch.from_numpy(x).to(dev)
        y, c = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        assert oracle.rel_l2(y.cpu().numpy(), oracle.fft(x)) <= 2e-6
        assert tf.counts_dict(c)["detected"] == 0
        tf.inject_arm(batch - 1, 3, 1, 27, dtype=dtype)
        y2, c2 = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        cd = tf.counts_dict(c2)
        assert cd["detected"] == 1 and cd["last_signal"] == batch - 1, cd
        assert torch.equal(y2, y) or oracle.rel_l2(y2.cpu().numpy(), oracle.fft(x)) <= 2e-6
    finally:
        tf.set_tuning(N, dtype, T=old[0], kappa=old[1])


def _restore_tuning():
    """Back to the package's tuning table (tests that pin routes call this)."""
    import os
    if os.path.exists(tf._lib.TUNING_PATH):
        tf.load_tuning(tf._lib.TUNING_PATH)


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
def test_two_pass_parity(dev, dtype):
    try:
        _two_pass_parity(dev, dtype)
    finally:
        for N in TWO_PASS[dtype]:
            tf.set_route(N, dtype, 0)
        _restore_tuning()


def _two_pass_parity(dev, dtype):
    for N in TWO_PASS[dtype]:
        # the ABFT modes give bit-identical outputs on one route; the tuning
        # table may give each mode its own, so pin the correcting mode's
        tf.set_route(N, dtype, tf.get_route(N, dtype, tf.FT_CORRECT))
        batch = max(3, (1 << 19) // N) + 1
        x = synth.signals(batch, N, seed=5000 + N, dtype=NPDT[dtype])
        xd = torch.from_numpy(x).to(dev)
        ref = oracle.fft(x, threads=8)
        y0, _ = tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=tf.FT_OFF)
        y0h = y0.cpu().numpy()
        assert oracle.rel_l2(y0h, ref) <= TOL[dtype], N
        assert _per_signal_rel(y0h, ref).max() <= TOL[dtype], N
        for ft in (tf.FT_DETECT, tf.FT_CORRECT):
            y, counts = tf.fft_c2c(xd, dir=tf.FORWARD, ft_mode=ft)
            c = tf.counts_dict(counts)
            assert c["detected"] == 0, (N, ft, c)
            assert torch.equal(y, y0), (N, ft)
        # inverse and in place
        yi, _ = tf.fft_c2c(xd, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT)
        assert oracle.rel_l2(yi.cpu().numpy(), oracle.fft(x, dir=+1, threads=8)) <= TOL[dtype], N
        xin = xd.clone()
        tf.fft_c2c(xin, dir=tf.FORWARD, ft_mode=tf.FT_CORRECT, out=xin)
        assert torch.equal(xin, y0), N


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
def test_two_pass_small_chunks(dev, dtype):
    # chunking of the batch must not change any output bit
    from paper_2412_05824_amd import _lib
    N = TWO_PASS[dtype][1]
    batch = 13
    x = synth.signals(batch, N, seed=6000, dtype=NPDT[dtype])
    xd = torch.from_numpy(x).to(dev)
    y_full, _ = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
    prec = 0 if dtype == torch.complex64 else 1
    sig_bytes = N * (8 if prec == 0 else 16)
    try:
        assert _lib.load().tfft_set_chunk(N, prec, 3 * sig_bytes) == 0
        y_chunk, c = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        assert torch.equal(y_full, y_chunk)
        assert tf.counts_dict(c)["detected"] == 0
        # an injection in the last chunk is located with its global index
        tf.inject_arm(batch - 2, 7, 1, 29 if prec == 0 else 61, dtype=dtype)
        y_inj, c2 = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        cd = tf.counts_dict(c2)
        assert cd["detected"] == 1 and cd["last_signal"] == batch - 2, cd
        assert oracle.rel_l2(y_inj.cpu().numpy()[batch - 2], oracle.fft(x[batch - 2])) <= TOL[dtype]
        assert oracle.rel_l2(y_inj[batch - 2].cpu().numpy(), y_full[batch - 2].cpu().numpy()) <= TOL[dtype]
    finally:
        _lib.load().tfft_set_chunk(N, prec, 128 << 20)


@pytest.mark.parametrize("dtype", DTYPES, ids=["fp32", "fp64"])
def test_two_pass_injection(dev, dtype):
    N = TWO_PASS[dtype][0]
    batch = 9
    nbits = 31 if dtype == torch.complex64 else 63
    rng = np.random.default_rng(99)
    for bit in [nbits - 1, nbits - 4, nbits - 9, nbits // 2, 3]:
        sig, elem, part = int(rng.integers(0, batch)), int(rng.integers(0, N)), int(rng.integers(0, 2))
        x, ref, yc, yh, c, delta = _inject_case(dev, dtype, N, batch, sig, elem, part, bit)
        per = _per_signal_rel(yh, ref)
        msg = f"N={N} bit={bit} sig={sig} elem={elem} counts={c} delta={delta:.3e}"
        assert per.max() <= TOL[dtype], msg + f" worst={per.max():.3e}"
        assert oracle.rel_l2(yh[sig], yc[sig]) <= TOL[dtype], msg
        if c["detected"]:
            assert c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == sig, msg
        else:
            assert delta <= TOL[dtype] * np.linalg.norm(ref[sig]), msg


@pytest.mark.parametrize("dtype,N", [(torch.complex64, n) for n in
                                     [64, 128, 256, 512, 1024, 2048, 4096, 8192, 1 << 14, 1 << 16]] +
                         [(torch.complex128, n) for n in [64, 256, 1024, 2048, 4096, 1 << 13, 1 << 16]],
                         ids=lambda v: str(v).replace("torch.complex64", "fp32").replace("torch.complex128", "fp64"))
def test_no_false_alarm_at_scale(dev, dtype, N):
    """Fault-free data count no detection also on batches of 2^26 elements
    (tens of thousands of workgroups, so races between waves of a workgroup
    would show), with the tuned route of each length."""
    g = torch.Generator(device=dev)
    g.manual_seed(N)
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    x = (torch.rand((1 << 26) // N, N, 2, dtype=rdt, device=dev, generator=g) * 2 - 1).view(dtype)
    x = x.view((1 << 26) // N, N)
    for ft in (tf.FT_DETECT, tf.FT_CORRECT):
        y, counts = tf.fft_c2c(x, ft_mode=ft)
        torch.cuda.synchronize()
        c = tf.counts_dict(counts)
        assert c["detected"] == 0 and c["uncorrectable"] == 0, (N, ft, c)
    del x, y


@pytest.mark.parametrize("N", [64, 1 << 16])
def test_batch_beyond_2_31_elements(dev, N):
    """A batch of 2^31 + 2^20 complex64 elements (16 GiB per buffer): element
    offsets past 2^31 must not wrap.  Signals on both sides of the 2^31
    boundary and the last one are checked against the oracle."""
    total = (1 << 31) + (1 << 20)
    batch = total // N
    g = torch.Generator(device=dev)
    g.manual_seed(N + 31)
    x = (torch.rand(batch, N, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(batch, N)
    y, counts = tf.fft_c2c(x, ft_mode=tf.FT_CORRECT)
    torch.cuda.synchronize()
    assert tf.counts_dict(counts)["detected"] == 0
    edge = (1 << 31) // N
    pick = [0, edge - 1, edge, edge + 1, batch - 1]
    xs = x[pick].cpu().numpy()
    ref = oracle.fft(xs)
    got = y[pick].cpu().numpy()
    for i, s in enumerate(pick):
        assert oracle.rel_l2(got[i], ref[i]) <= 2e-6, (N, s)
    del x, y
    torch.cuda.empty_cache()
