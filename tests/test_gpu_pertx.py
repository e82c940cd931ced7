"""Per-transaction detection with delayed batched correction (Sec. 4.1
"Delayed Batched Correction"; Sec. 4.3 multi-transaction groups), on the GPU.

Each signal of a group is checked against a threshold from its own input
energy; a faulty one is noted, the group carries on, and at its end every
noted signal is repaired from the right-side sums of the transactions before
the next faulty one (or of the whole group), oldest first.  Reference
semantics: oracle.abft_model.abft_group_per_transaction.

Checked here, in fp32 at groups of up to 16 signals (more than the
group-level check allows under the fp32 tolerance):
  * a flip of any bit in any transaction of a group, in a single-pass plan
    whose slot is below a wave, one spanning several waves, and both passes
    of a two-pass transform: significant flips detected and repaired, every
    signal (hit or not) within the tolerance of its fault-free output, the
    others bit-identical;
  * two faults in one group (sequential errors): both repaired;
  * in place, where the input sums live in registers: one fault repaired,
    two counted uncorrectable;
  * the route reports the granularity and the transactions per group it runs.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from groups import group_of

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = 2e-6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _with_T(N, T, fn, dtype=torch.complex64, gran=1):
    old = tf.get_tuning(N, dtype)
    old_gran = tf.route_info(N, dtype)["gran"]
    tf.set_tuning(N, dtype, T=T)
    tf.set_granularity(N, dtype, gran)
    try:
        return fn()
    finally:
        tf.set_tuning(N, dtype, T=old[0], kappa=old[1])
        tf.set_granularity(N, dtype, old_gran)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_route_reports_granularity(dev):
    """The route reports the granularity of the shipped tuning table (none
    without ABFT), follows tfft_set_granularity, and reduces a T beyond what
    the plan keeps when checking per transaction."""
    import json
    table = json.load(open(tf._lib.TUNING_PATH))
    for e in table["entries"]:
        if e["ft_mode"] != 2:
            continue
        dtype = torch.complex64 if e["precision"] == "fp32" else torch.complex128
        assert tf.route_info(e["N"], dtype)["gran"] == e["gran"], e
        assert tf.route_info(e["N"], dtype, ft_mode=0)["gran"] == 0
    for gran in (0, 1):
        assert _with_T(1024, 4, lambda: tf.route_info(1024, torch.complex128)["gran"],
                       dtype=torch.complex128, gran=gran) == gran
    info = _with_T(256, 32, lambda: tf.route_info(256, torch.complex64))
    assert 1 <= info["T"] <= 16, info


@pytest.mark.parametrize("N", [256, 4096, 1 << 16], ids=["256-subwave", "4096-multiwave", "2^16-twopass"])
def test_every_bit_any_transaction_per_tx(dev, N):
    def body():
        info = tf.route_info(N, torch.complex64)
        T = info["T"]
        assert info["gran"] == 1 and T >= 4, info
        # three rounds of full groups over the workgroups' slots
        batch = 3 * T * (info["slots0"] if info["passes"] == 1 else 1)
        g0 = group_of(0, batch, info)
        tail = group_of(batch - 1, batch, info)
        assert len(g0) == T and len(tail) == T and g0 != tail, (g0, tail, info)
        # transactions 0, middle and last of a group, and of another group
        targets = [g0[0], g0[T // 2], g0[T - 1], tail[0], tail[-1]]
        x = synth.signals(batch, N, seed=9500 + N)
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        yc = y0.cpu().numpy()
        rng = np.random.default_rng(N)
        passes = [(0, -1)] if info["passes"] == 1 else [(0, -1), (1, -1), (0, 0)]
        n_sig = 0
        for trial in range(24):
            pass_, stage = passes[trial % len(passes)]
            sig = targets[trial % 5]
            bit = int(rng.integers(0, 31))
            elem, part = int(rng.integers(0, N)), int(rng.integers(0, 2))
            tf.inject_arm(sig, elem, part, bit, pass_=pass_, stage=stage)
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
            c = tf.counts_dict(counts)
            msg = f"N={N} T={T} sig={sig} bit={bit} pass={pass_} stage={stage} {c}"
            yh = y.cpu().numpy()
            err = np.linalg.norm(yh - yc, axis=1) / np.linalg.norm(yc, axis=1)
            assert err.max() <= TOL, msg + f" rel {err.max():.3e} at {err.argmax()}"
            assert c["uncorrectable"] == 0, msg
            if c["detected"]:
                n_sig += 1
                assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == sig, msg
            keep = np.ones(batch, bool)
            keep[sig] = False
            assert np.array_equal(yh[keep], yc[keep]), msg
            if bit >= 28:   # exponent flips are far above any threshold
                assert c["detected"] == 1, msg
        assert n_sig >= 8, n_sig
        ref = oracle.fft(x[[0, batch - 1]], threads=8)
        assert oracle.rel_l2(yh[[0, batch - 1]], ref) <= TOL
    _with_T(N, 16, body)


@pytest.mark.parametrize("N", [512, 4096, 1 << 16])
def test_two_faults_in_one_group_both_repaired(dev, N):
    """Sequential errors (Sec. 4.1): the older fault is corrected from the
    sums of the transactions before the newer one, the newer from the whole
    group's, with the older already repaired."""
    def body():
        info = tf.route_info(N, torch.complex64)
        T = info["T"]
        batch = 2 * T * (info["slots0"] if info["passes"] == 1 else 1)   # two rounds of full groups
        x = synth.signals(batch, N, seed=9600 + N)
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        yc = y0.cpu().numpy()
        ga, gb = group_of(1, batch, info), group_of(batch - 1, batch, info)
        assert len(ga) == T and len(gb) >= 2, (ga, gb)
        # two transactions of one group: neighbours, first and last, and in
        # the last group
        for s1, s2, bit in [(ga[1], ga[2], 25), (ga[0], ga[-1], 30), (gb[0], gb[-1], 22)]:
            tf.inject_arm(s1, N // 3, 0, bit, signal2=s2)
            y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
            c = tf.counts_dict(counts)
            msg = f"N={N} T={T} faults at {s1},{s2} bit={bit} {c}"
            assert c["detected"] == 2 and c["corrected"] + c["rebuilt"] == 2 and c["uncorrectable"] == 0, msg
            yh = y.cpu().numpy()
            for s in (s1, s2):
                assert _rel(yh[s], yc[s]) <= TOL, msg + f" signal {s}"
            keep = np.ones(batch, bool)
            keep[[s1, s2]] = False
            assert np.array_equal(yh[keep], yc[keep]), msg
    _with_T(N, 4, body)


def test_two_faults_in_one_column_pass_group(dev):
    N = 1 << 16
    def body():
        info = tf.route_info(N, torch.complex64)
        T = info["T"]
        batch = T   # one group of the column pass
        assert group_of(0, batch, info) == list(range(T))
        x = synth.signals(batch, N, seed=9650)
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        yc = y0.cpu().numpy()
        tf.inject_arm(0, 777, 1, 27, pass_=0, stage=0, signal2=T - 1)
        y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        c = tf.counts_dict(counts)
        assert c["detected"] == 2 and c["corrected"] + c["rebuilt"] == 2, c
        yh = y.cpu().numpy()
        assert max(_rel(yh[s], yc[s]) for s in range(batch)) <= TOL, c
    _with_T(N, 4, body)


def test_in_place_one_fault_repaired_two_not(dev):
    N, T = 1024, 4
    def body():
        batch = 2 * T
        info = tf.route_info(N, torch.complex64)
        pair = group_of(1, batch, info)[:2]
        x = synth.signals(batch, N, seed=9700)
        y0, _ = tf.fft_c2c(torch.from_numpy(x).to(dev), ft_mode=tf.FT_OFF)
        yc = y0.cpu().numpy()
        xd = torch.from_numpy(x).to(dev)
        tf.inject_arm(2, 100, 0, 29)
        y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT, out=xd)
        c = tf.counts_dict(counts)
        assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1, c
        assert _rel(y.cpu().numpy()[2], yc[2]) <= TOL
        xd = torch.from_numpy(x).to(dev)
        tf.inject_arm(pair[0], 100, 0, 29, signal2=pair[1])
        y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT, out=xd)
        c = tf.counts_dict(counts)
        assert c["detected"] == 2 and c["uncorrectable"] == 2 and c["corrected"] + c["rebuilt"] == 0, c
    _with_T(N, T, body)


def test_group_granularity_still_locates(dev):
    """fp32 with the group-level check (location code D1/D0) at T = 2, the
    largest the fp32 tolerance allows for it: an exponent flip is located
    and corrected."""
    N = 512
    def body():
        batch = 8
        x = synth.signals(batch, N, seed=9750)
        xd = torch.from_numpy(x).to(dev)
        y0, _ = tf.fft_c2c(xd, ft_mode=tf.FT_OFF)
        tf.inject_arm(5, 33, 1, 29)
        y, counts = tf.fft_c2c(xd, ft_mode=tf.FT_CORRECT)
        c = tf.counts_dict(counts)
        assert c["detected"] == 1 and c["corrected"] + c["rebuilt"] == 1 and c["last_signal"] == 5, c
        assert _rel(y.cpu().numpy()[5], y0.cpu().numpy()[5]) <= TOL
    assert _with_T(N, 2, lambda: tf.route_info(N, torch.complex64)["gran"], gran=0) == 0
    _with_T(N, 2, body, gran=0)


def test_no_false_alarm_per_tx_at_T16(dev):
    for N in (64, 2048, 1 << 18):
        def body():
            batch = (1 << 24) // N
            g = torch.Generator(device=dev)
            g.manual_seed(9800 + N)
            x = (torch.rand(batch * N, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(batch, N)
            y, counts = tf.fft_c2c(x, ft_mode=tf.FT_CORRECT)
            assert tf.counts_dict(counts)["detected"] == 0, N
        _with_T(N, 16, body)
