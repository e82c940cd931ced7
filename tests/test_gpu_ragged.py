"""GPU parity of ragged batches (mixed lengths in one call) against the oracle.

Each signal of a ragged batch is transformed as tfft_c2c would (Sec. 2.2),
under the same ABFT protection (Sec. 4): relative L2 <= 2e-6 per signal
against the fp64 oracle.  The persistent single launch and the per-size
launches run the same kernel bodies on the same data, so their outputs and
counters agree bit for bit; ABFT on changes no output bit when no fault
occurs; an injected flip (Sec. 5.3 protocol) in any signal is detected,
located and corrected.  The persistent launch replays from a captured graph.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tf = pytest.importorskip("paper_2412_05824_amd")

TOL = 2e-6
MODES = ("persistent", "per_size")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ragged_input(sizes, seed):
    total = int(np.sum(sizes))
    return synth.signals(1, total, seed=seed, dtype=np.complex64).reshape(-1)


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))])


def _oracle_ragged(x, sizes, dir=-1, scale=None, only=None):
    """Per-signal oracle transforms (dict index -> complex128), grouped by length."""
    off = _offsets(sizes)
    idx = range(len(sizes)) if only is None else only
    by_len = {}
    for i in idx:
        by_len.setdefault(int(sizes[i]), []).append(i)
    out = {}
    for n, ids in by_len.items():
        stack = np.stack([x[off[i]:off[i] + n] for i in ids])
        ref = oracle.fft(stack, dir=dir, scale=scale, threads=8)
        for j, i in enumerate(ids):
            out[i] = ref[j]
    return out


def _small_sizes(seed=11):
    # every length of the menu at least once (single-pass and two-pass routes,
    # groups of T = 2 with an odd tail), then a seeded draw, shuffled
    menu = list(synth.RAGGED_SIZES)
    sizes = menu + [64, 64, 64, 128, 192, 192] + list(synth.ragged_sizes(40, seed=seed))
    rng = synth.rng(seed)
    rng.shuffle(sizes)
    return [int(s) for s in sizes]


def _plan(sizes, dev, window=0, waves=3):
    """A plan built under a schedule (window = 0: flat workspace; waves = 3:
    the persistent kernel held to three workgroups per CU, the default;
    0: the compiler's register budget)."""
    tf.ragged_set_schedule(window, 0, waves)
    try:
        return tf.RaggedPlan(sizes, device=dev)
    finally:
        tf.ragged_set_schedule(0, 0, 3)


# (window, waves): flat workspace; a ring of two 2^18-element halves (many
# batches, so column passes of later batches wait for earlier row passes);
# the compiler's register budget instead of three workgroups per CU
SCHEDULES = [(0, 3), (1 << 18, 3), (0, 0)]
WINDOWS = [0, 1 << 18]


def _check_signals(y, x_host, sizes, refs, tol=TOL):
    off = _offsets(sizes)
    worst = 0.0
    for i, ref in refs.items():
        got = y[off[i]:off[i] + sizes[i]]
        e = oracle.rel_l2(got, ref)
        worst = max(worst, e)
        assert e <= tol, f"signal {i} (N={sizes[i]}): rel L2 {e:.3e}"
    return worst


@pytest.mark.parametrize("window,waves", SCHEDULES)
@pytest.mark.parametrize("ft", [tf.FT_OFF, tf.FT_CORRECT])
def test_ragged_parity_and_modes(dev, ft, window, waves):
    sizes = _small_sizes()
    x_host = _ragged_input(sizes, seed=101)
    x = torch.from_numpy(x_host).to(dev)
    plan = _plan(sizes, dev, window, waves)
    info = plan.info()
    assert info["signals"] == len(sizes) and info["total"] == x.numel()
    assert (info["batches"] > 2) == (window > 0), info
    outs = {}
    for mode in MODES:
        counts = tf.new_counts(dev)
        y, _ = plan(x, ft_mode=ft, counts=counts, mode=mode)
        torch.cuda.synchronize()
        outs[mode] = y.cpu().numpy()
        c = tf.counts_dict(counts)
        assert c["detected"] == 0 and c["uncorrectable"] == 0, (mode, c)
    assert np.array_equal(outs["persistent"].view(np.uint32), outs["per_size"].view(np.uint32))
    refs = _oracle_ragged(x_host, sizes)
    worst = _check_signals(outs["persistent"], x_host, sizes, refs)
    print(f"ragged {len(sizes)} signals ft={ft}: worst rel L2 {worst:.3e}")
    st = plan.info(device_state=True)
    assert st["err_launches"] == 0 and st["queue_next"] == 0


def test_ragged_abft_changes_no_bit(dev):
    sizes = _small_sizes(seed=12)
    x = torch.from_numpy(_ragged_input(sizes, seed=102)).to(dev)
    plan = tf.RaggedPlan(sizes, device=dev)
    y0, _ = plan(x, ft_mode=tf.FT_OFF)
    y1, c1 = plan(x, ft_mode=tf.FT_DETECT)
    y2, c2 = plan(x, ft_mode=tf.FT_CORRECT)
    torch.cuda.synchronize()
    b0 = y0.cpu().numpy().view(np.uint32)
    assert np.array_equal(b0, y1.cpu().numpy().view(np.uint32))
    assert np.array_equal(b0, y2.cpu().numpy().view(np.uint32))
    assert tf.counts_dict(c1)["detected"] == 0 and tf.counts_dict(c2)["detected"] == 0


@pytest.mark.parametrize("mode", MODES)
def test_ragged_inverse_and_unit_scale(dev, mode):
    sizes = _small_sizes(seed=13)
    x_host = _ragged_input(sizes, seed=103)
    x = torch.from_numpy(x_host).to(dev)
    plan = tf.RaggedPlan(sizes, device=dev)
    yi, c = plan(x, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT, mode=mode)
    yu, cu = plan(x, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT, unit_scale=True, mode=mode)
    torch.cuda.synchronize()
    assert tf.counts_dict(c)["detected"] == 0 and tf.counts_dict(cu)["detected"] == 0
    _check_signals(yi.cpu().numpy(), x_host, sizes, _oracle_ragged(x_host, sizes, dir=+1))
    _check_signals(yu.cpu().numpy(), x_host, sizes, _oracle_ragged(x_host, sizes, dir=+1, scale=1.0))
    # forward then inverse returns the input
    yf, _ = plan(x, ft_mode=tf.FT_CORRECT, mode=mode)
    back, _ = plan(yf, dir=tf.INVERSE, ft_mode=tf.FT_CORRECT, mode=mode)
    torch.cuda.synchronize()
    off = _offsets(sizes)
    bk = back.cpu().numpy()
    for i, n in enumerate(sizes):
        assert oracle.rel_l2(bk[off[i]:off[i] + n], x_host[off[i]:off[i] + n]) <= 2 * TOL


# (length, bit): single-pass groups of T = 2 and T = 1, two-pass lengths
INJ = [(64, 27), (192, 22), (3072, 30), (4096, 26), (6144, 29), (196608, 28), (1 << 16, 23)]


@pytest.mark.parametrize("mode", MODES + ("windowed", "w0"))
@pytest.mark.parametrize("n,bit", INJ)
def test_ragged_injection_corrected(dev, mode, n, bit):
    sizes = _small_sizes(seed=14)
    x_host = _ragged_input(sizes, seed=104)
    x = torch.from_numpy(x_host).to(dev)
    plan = _plan(sizes, dev, WINDOWS[1] if mode == "windowed" else 0, 0 if mode == "w0" else 3)
    mode = "persistent" if mode in ("windowed", "w0") else mode
    clean, _ = plan(x, ft_mode=tf.FT_CORRECT, mode=mode)
    cands = [i for i, s in enumerate(sizes) if s == n]
    g = synth.rng(1000 + n + bit)
    sig = int(cands[int(g.integers(0, len(cands)))])
    elem = int(g.integers(0, n))
    part = int(g.integers(0, 2))
    counts = tf.new_counts(dev)
    tf.inject_arm(sig, elem, part, bit)
    y, _ = plan(x, ft_mode=tf.FT_CORRECT, counts=counts, mode=mode)
    torch.cuda.synchronize()
    c = tf.counts_dict(counts)
    assert c["detected"] == 1 and c["uncorrectable"] == 0, c
    assert c["corrected"] + c["rebuilt"] == 1, c
    assert c["last_signal"] == sig, c
    off = _offsets(sizes)
    yh = y.cpu().numpy()
    ch = clean.cpu().numpy()
    ref = _oracle_ragged(x_host, sizes, only=[sig])[sig]
    assert oracle.rel_l2(yh[off[sig]:off[sig] + n], ref) <= TOL
    # every other signal is untouched
    mask = np.ones(yh.shape[0], dtype=bool)
    mask[off[sig]:off[sig] + n] = False
    assert np.array_equal(yh[mask].view(np.uint32), ch[mask].view(np.uint32))


@pytest.mark.parametrize("window,waves", SCHEDULES)
def test_ragged_graph_replay(dev, window, waves):
    sizes = _small_sizes(seed=15)
    x_host = _ragged_input(sizes, seed=105)
    x = torch.from_numpy(x_host).to(dev)
    plan = _plan(sizes, dev, window, waves)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan(x, out=y, ft_mode=tf.FT_CORRECT, counts=counts)   # warm up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan(x, out=y, ft_mode=tf.FT_CORRECT, counts=counts)
    torch.cuda.synchronize()
    for r in range(4):
        # new data each replay, eager work of the same plan in between
        fresh = _ragged_input(sizes, seed=200 + r)
        x.copy_(torch.from_numpy(fresh).to(dev))
        eager, _ = plan(x, ft_mode=tf.FT_CORRECT, mode="per_size")
        counts.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint32), eager.cpu().numpy().view(np.uint32)), r
        assert tf.counts_dict(counts)["detected"] == 0
    st = plan.info(device_state=True)
    assert st["err_launches"] == 0 and st["queue_next"] == 0
    refs = _oracle_ragged(fresh, sizes, only=range(0, len(sizes), 7))
    _check_signals(y.cpu().numpy(), fresh, sizes, refs)


def test_ragged_edges(dev):
    # empty list
    empty = tf.RaggedPlan([], device=dev)
    z = torch.empty(0, dtype=torch.complex64, device=dev)
    empty(z)
    # one signal of each route
    for n in (64, 4096, 196608):
        x_host = _ragged_input([n], seed=n)
        x = torch.from_numpy(x_host).to(dev)
        p = tf.RaggedPlan([n], device=dev)
        y, c = p(x)
        torch.cuda.synchronize()
        assert oracle.rel_l2(y.cpu().numpy(), oracle.fft(x_host[None])[0]) <= TOL
    # unsupported length
    with pytest.raises(tf.TfftError):
        tf.RaggedPlan([64, 100], device=dev)
    sizes = _small_sizes(seed=16)
    x = torch.from_numpy(_ragged_input(sizes, seed=106)).to(dev)
    p = tf.RaggedPlan(sizes, device=dev)
    # in place: allowed without correction, refused with it
    ref, _ = p(x, ft_mode=tf.FT_DETECT)
    xi = x.clone()
    p(xi, out=xi, ft_mode=tf.FT_DETECT)
    torch.cuda.synchronize()
    assert np.array_equal(xi.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32))
    with pytest.raises(tf.TfftError):
        p(xi, out=xi, ft_mode=tf.FT_CORRECT)


@pytest.mark.parametrize("window,waves", [(0, 3), (1 << 23, 3), (0, 0)])
def test_ragged_full_workload(dev, window, waves):
    """The 10,000-signal workload (lengths drawn from the 22-length menu),
    persistent vs per-size bit for bit, sampled signals against the oracle."""
    sizes = [int(s) for s in synth.ragged_sizes(10000, seed=5)]
    x_host = _ragged_input(sizes, seed=2005)
    x = torch.from_numpy(x_host).to(dev)
    plan = _plan(sizes, dev, window, waves)
    cp, cs = tf.new_counts(dev), tf.new_counts(dev)
    yp, _ = plan(x, ft_mode=tf.FT_CORRECT, counts=cp, mode="persistent")
    ys, _ = plan(x, ft_mode=tf.FT_CORRECT, counts=cs, mode="per_size")
    torch.cuda.synchronize()
    assert tf.counts_dict(cp)["detected"] == 0 and tf.counts_dict(cs)["detected"] == 0
    assert torch.equal(yp.view(torch.float32), ys.view(torch.float32))
    pick = [int(i) for i in synth.sample_indices(len(sizes), 24, seed=6)]
    refs = _oracle_ragged(x_host, sizes, only=pick)
    off = _offsets(sizes)
    for i in pick:
        got = yp[int(off[i]):int(off[i + 1])].cpu().numpy()
        e = oracle.rel_l2(got, refs[i])
        assert e <= TOL, (i, sizes[i], e)
    st = plan.info(device_state=True)
    assert st["err_launches"] == 0 and st["queue_next"] == 0


@pytest.mark.parametrize("window", [0, 1 << 21])
def test_ragged_wait_bound_reported_then_clean(dev, window):
    """The host forces every bounded wait of one persistent launch to give
    up (each wait needs one more finished item than exist and polls at most
    64 times): the launch still drains, counts one schedule error and leaves
    its counters zeroed, so the next launch is bit-identical to the per-size
    launches with no error.  Every kernel exits normally."""
    from paper_2412_05824_amd import _lib
    sizes = [1 << 14] * 6 + [3 << 14] * 3 + [1 << 16] * 3 + [256] * 40 + [1 << 17]
    x = torch.from_numpy(_ragged_input(sizes, seed=301)).to(dev)
    plan = _plan(sizes, dev, window, 3)
    lib = _lib.load()
    ref, _ = plan(x, ft_mode=tf.FT_CORRECT, mode="per_size")
    counts = tf.new_counts(dev)
    assert lib.tfft_ragged_test_wait(64, 1) == 0
    try:
        plan(x, ft_mode=tf.FT_CORRECT, counts=counts, mode="persistent")
        torch.cuda.synchronize()
    finally:
        lib.tfft_ragged_test_wait(0, 0)
    c = tf.counts_dict(counts)
    assert c["sched_errors"] == 1, c
    st = plan.info(device_state=True)
    assert st["err_launches"] == 1 and st["queue_next"] == 0, st
    counts2 = tf.new_counts(dev)
    y2, _ = plan(x, ft_mode=tf.FT_CORRECT, counts=counts2, mode="persistent")
    torch.cuda.synchronize()
    c2 = tf.counts_dict(counts2)
    assert c2["sched_errors"] == 0 and c2["detected"] == 0, c2
    assert torch.equal(y2.view(torch.float32), ref.view(torch.float32))
    assert plan.info(device_state=True)["err_launches"] == 1
