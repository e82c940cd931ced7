"""Pins for the CPU ABFT reference model (TurboFFT Sec. 2.2, Sec. 4.1-4.3).

The checks come from the mathematics of the paper's equations, not from the
model's own code: closed forms and brute-force sums written here, the error
propagation of real FFT stage orders written here (radix-2 DIT and the radix-16
Stockham order the GPU kernels use), the location identity, the correction
identity of Eq. 5, and finite differences for the gradient.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import abft_model as am
import synth


def brute_left(N, M, dir=-1):
    """(e^T W)_n = sum_k e_k w_N^{dir k n}, summed term by term."""
    k = np.arange(N)
    e = np.exp(-2j * np.pi * (k % M) / M)
    out = np.empty(N, complex)
    for n in range(N):
        out[n] = np.sum(e * np.exp(dir * 2j * np.pi * ((k * n) % N) / N))
    return out


@pytest.mark.parametrize("N", [8, 64, 96, 1024, 6144, 8192, 16384])
def test_left_vector_cotangent_form(N):
    """The streaming single-pass kernels encode with a real table: with
    w_M w_N^n = exp(-i theta_n), 1 / (1 - exp(-i theta)) = (1 - i cot(theta/2)) / 2,
    so a_n = c2 (1 - i cot(theta_n / 2)), c2 = (1 - w_M^N) / 2, and
    p = a^T x = c2 (S - i C) with S = sum x_n, C = sum cot_n x_n.  Checked
    against e^T W summed term by term (small N) and the oracle's transform
    of e (large N); theta_n / 2 = pi k / (M N), k = (N + M n) mod (M N) > 0."""
    M = am.choose_M(N)
    n = np.arange(N)
    k = (N + M * n) % (M * N)
    assert k.min() > 0
    cot = np.cos(np.pi * k / (M * N)) / np.sin(np.pi * k / (M * N))
    c2 = (1 - np.exp(-2j * np.pi * N / M)) / 2
    ref = brute_left(N, M) if N <= 1024 else am.left_vector(N, M)
    np.testing.assert_allclose(c2 * (1 - 1j * cot), ref, rtol=0, atol=1e-10 * N)
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    S, C = x.sum(), (cot * x).sum()
    p = c2 * complex(S.real + C.imag, S.imag - C.real)
    assert abs(p - ref @ x) <= 1e-10 * N * np.linalg.norm(x)


@pytest.mark.parametrize("N", [1024, 6144, 8192, 16384])
def test_cotangent_form_rounding_in_fp32(N):
    """Reading 27's claim that the cotangent form rounds like the complex
    table: the input checksum p = a^T x computed in complex64 from each
    table, rounded once, over 20 seeded U[-1,1) signals.  Both errors stay a
    fraction of the fp32 threshold tau (kappa = 8) and the cotangent form's
    is within 1.5x of the complex table's."""
    M = am.choose_M(N)
    a = am.left_vector(N, M)
    n = np.arange(N)
    k = (N + M * n) % (M * N)
    cot32 = (np.cos(np.pi * k / (M * N)) / np.sin(np.pi * k / (M * N))).astype(np.float32)
    c2 = np.complex64((1 - np.exp(-2j * np.pi * N / M)) / 2)
    a32 = a.astype(np.complex64)
    worst_c = worst_t = 0.0
    for seed in range(20):
        rng = np.random.default_rng(seed)
        x = (rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)).astype(np.complex64)
        p = a @ x.astype(np.complex128)
        tau = am.threshold(N, float(np.sum(np.abs(x.astype(np.complex128)) ** 2)), "fp32", 8.0)
        pc = (a32 * x).sum(dtype=np.complex64)
        S, C = x.sum(dtype=np.complex64), (cot32 * x).sum(dtype=np.complex64)
        pt = c2 * np.complex64(complex(S.real + C.imag, S.imag - C.real))
        worst_c = max(worst_c, abs(pc - p) / tau)
        worst_t = max(worst_t, abs(pt - p) / tau)
    assert worst_c < 0.5 and worst_t < 0.5, (worst_c, worst_t)
    assert worst_t <= 1.5 * worst_c, (worst_c, worst_t)


@pytest.mark.parametrize("N,M", [(8, 3), (64, 3), (256, 3), (12, 5), (96, 5), (48, 7), (1024, 5)])
def test_left_vector_closed_form_and_norm(N, M):
    for d in (-1, +1):
        ref = brute_left(N, M, d)
        np.testing.assert_allclose(am.left_vector(N, M, d), ref, rtol=0, atol=1e-10 * N)
        np.testing.assert_allclose(am.left_vector_closed_form(N, M, d), ref, rtol=0, atol=1e-10 * N)
        # ||e^T W||_2 = N (Parseval with ||e||^2 = N)
        assert abs(np.linalg.norm(am.left_vector(N, M, d)) - N) <= 1e-9 * N


def test_m3_degenerates_when_3_divides_N():
    # with 3 | N, w_3^N = 1 and e^T W collapses onto a single index, like the
    # all-ones vector; the model then switches to M = 5
    for N in (12, 48, 96, 3 << 10):
        a3 = brute_left(N, 3)
        assert np.sum(np.abs(a3) > 1e-6 * N) == 1
        assert am.choose_M(N) == 5
        assert np.min(np.abs(am.left_vector(N, 5))) > 0.1
    for N in (64, 1 << 12):
        assert am.choose_M(N) == 3
        assert np.min(np.abs(am.left_vector(N, 3))) > 0.1


def test_checksum_identity_fault_free():
    # (e^T W) x = e^T (W x)  (Eq. 1-2), two-side form Eq. 4-5
    N, G = 256, 8
    X = synth.signals(G, N, seed=5, dtype=np.complex128)
    Y = oracle.fft(X)
    cs = am.group_checksums(X, Y, 3)
    scale = math.sqrt(N * cs["nu"])
    assert abs(cs["s_out"] - cs["s_in"]) <= 1e-13 * scale
    assert abs(cs["l_out"] - cs["l_in"]) <= 1e-12 * scale
    np.testing.assert_allclose(oracle.fft(cs["x_s"]), cs["y_s"], rtol=0, atol=1e-12 * scale)


# --- stage-ordered FFTs written here to inject errors between stages -------

def dit_radix2_with_fault(x, stage, pos, eps):
    """Iterative radix-2 DIT; adds eps to element pos after `stage` butterflies."""
    N = len(x)
    lg = int(math.log2(N))
    idx = np.array([int(format(i, f"0{lg}b")[::-1], 2) for i in range(N)])
    a = np.array(x, complex)[idx]
    if stage == 0:
        a[pos] += eps
    m = 1
    for s in range(1, lg + 1):
        w = np.exp(-2j * np.pi * np.arange(m) / (2 * m))
        for start in range(0, N, 2 * m):
            u = a[start:start + m].copy()
            v = a[start + m:start + 2 * m] * w
            a[start:start + m] = u + v
            a[start + m:start + 2 * m] = u - v
        m *= 2
        if s == stage:
            a[pos] += eps
    return a


def stockham_with_fault(x, radices, stage, pos, eps):
    """Stockham autosort: stage s combines L = prod(radices[:s]) into L*R.
    Adds eps to buffer element pos after stage `stage` (0 = on the input)."""
    N = len(x)
    a = np.array(x, complex)
    if stage == 0:
        a[pos] += eps
    L = 1
    for s, R in enumerate(radices, start=1):
        out = np.empty_like(a)
        F = np.exp(-2j * np.pi * np.outer(np.arange(R), np.arange(R)) / R)
        for beta in range(N // R):
            k, g = beta % L, beta // L
            v = a[beta + np.arange(R) * (N // R)] * np.exp(-2j * np.pi * np.arange(R) * k / (L * R))
            out[g * L * R + k + np.arange(R) * L] = F @ v
        a = out
        L *= R
        if s == stage:
            a[pos] += eps
    return a


def _d0_single(x, y_faulty, M):
    N = len(x)
    cs = am.group_checksums(x[None, :], y_faulty[None, :], M)
    return cs["s_out"] - cs["s_in"]


@pytest.mark.parametrize("N", [16, 64])
def test_detection_bound_radix2_every_stage_and_position(N):
    # any single additive fault eps between stages gives |D0| >= |eps| |1 - w_M^N| / 2
    x = synth.signals(1, N, seed=N, dtype=np.complex128)[0]
    np.testing.assert_allclose(dit_radix2_with_fault(x, -1, 0, 0), np.fft.fft(x), atol=1e-12)
    M = 3
    bound = abs(1 - np.exp(-2j * np.pi * N / M)) / 2
    eps = 1e-3 * (0.6 - 0.8j)
    lg = int(math.log2(N))
    worst = np.inf
    for stage in range(lg + 1):
        for pos in range(N):
            y = dit_radix2_with_fault(x, stage, pos, eps)
            worst = min(worst, abs(_d0_single(x, y, M)) / abs(eps))
    assert worst >= bound * (1 - 1e-6)
    assert worst <= bound * 1.5   # the bound is attained up to a small factor


def test_detection_bound_stockham_radix16():
    N, radices = 256, [16, 16]
    x = synth.signals(1, N, seed=3, dtype=np.complex128)[0]
    np.testing.assert_allclose(stockham_with_fault(x, radices, -1, 0, 0), np.fft.fft(x), atol=1e-11)
    for M in (3, 5):
        bound = abs(1 - np.exp(-2j * np.pi * N / M)) / 2
        eps = 2e-3 * (1 + 0.5j)
        worst = np.inf
        for stage in range(len(radices) + 1):
            for pos in range(N):
                y = stockham_with_fault(x, radices, stage, pos, eps)
                worst = min(worst, abs(_d0_single(x, y, M)) / abs(eps))
        assert worst >= bound * (1 - 1e-6)


def test_ones_vector_misses_faults():
    # Sec. 2.2: the all-ones vector misses some propagated faults; w_3 misses none
    N = 16
    x = synth.signals(1, N, seed=1, dtype=np.complex128)[0]
    eps = 1e-2
    missed_ones = missed_w3 = 0
    for stage in range(int(math.log2(N)) + 1):
        for pos in range(N):
            y = dit_radix2_with_fault(x, stage, pos, eps)
            y0 = np.fft.fft(x)
            d_ones = np.sum(y) - np.sum(y0)
            missed_ones += abs(d_ones) < 1e-9
            missed_w3 += abs(_d0_single(x, y, 3)) < 1e-9
    assert missed_ones > 0
    assert missed_w3 == 0


def test_location_identity():
    # D1 / D0 = b* + 1 for one fault in signal b* (location weights 1, 2, ...)
    N, G = 64, 8
    X = synth.signals(G, N, seed=9, dtype=np.complex128)
    Y = oracle.fft(X)
    for bstar in range(G):
        for stage in (0, 3, 6):
            Yf = Y.copy()
            Yf[bstar] = dit_radix2_with_fault(X[bstar], stage, (5 * bstar + 1) % N, 0.7 - 0.2j)
            cs = am.group_checksums(X, Yf, 3)
            r = (cs["l_out"] - cs["l_in"]) / (cs["s_out"] - cs["s_in"])
            assert abs(r - (bstar + 1)) < 1e-9


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_correction_restores_fault_free_output(precision):
    N, G = 128, 8
    X = synth.signals(G, N, seed=21, dtype=np.complex128)
    Y = oracle.fft(X)
    # fault-free group is clean
    assert am.abft_group(X, Y, precision)["action"] == "clean"
    for bstar, stage in [(0, 7), (3, 2), (7, 0)]:
        Yf = Y.copy()
        Yf[bstar] = dit_radix2_with_fault(X[bstar], stage, 17, 0.05 + 0.3j)
        r = am.abft_group(X, Yf, precision)
        assert r["action"] == "corrected"
        assert r["b"] == bstar
        # Eq. 5: W(Xe) - Y'e = -(fault), so the corrected output is the DFT
        assert oracle.rel_l2(r["Y"], Y) < 1e-13


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bit_flip_paths(precision):
    # An undetected flip changes one signal by at most tau, i.e. by a relative
    # kappa * u * sqrt(G log2 N) of its norm: in fp32 that stays below 2e-6 only
    # for small kappa * sqrt(G log2 N), which bounds the group size G.
    N = 256
    G, kappa = (4, 4.0) if precision == "fp32" else (8, 32.0)
    dt = np.complex64 if precision == "fp32" else np.complex128
    X = synth.signals(G, N, seed=33, dtype=dt).astype(np.complex128)
    Y = oracle.fft(X).astype(dt).astype(np.complex128)   # outputs as stored
    nbits = 31 if precision == "fp32" else 63
    tol = 2e-6 if precision == "fp32" else 1e-13
    kinds = set()
    for bit in range(nbits):
        for part in (0, 1):
            Yf = Y.copy()
            b, k = bit % G, (7 * bit + part) % N
            Yf[b, k] = am.flip_bit(complex(Y[b, k]), part, bit, precision)
            delta = abs(Yf[b, k] - Y[b, k])
            r = am.abft_group(X, Yf, precision, kappa=kappa)
            kinds.add(r["action"])
            if r["action"] == "clean":
                # undetected flips are below the threshold and harmless
                assert delta <= r["tau"]
                assert oracle.rel_l2(Yf[b], Y[b]) < tol
            else:
                assert r["action"] in ("corrected", "rebuilt")
                assert r["b"] == b
                assert oracle.rel_l2(r["Y"][b], Y[b]) < tol
            if np.isfinite(delta) and delta > 4 * r["tau"]:
                assert r["action"] != "clean"
    assert {"clean", "corrected", "rebuilt"} <= kinds


def test_non_finite_and_two_faults():
    N, G = 64, 4
    X = synth.signals(G, N, seed=2, dtype=np.complex128)
    Y = oracle.fft(X)
    Yf = Y.copy()
    Yf[2, 5] = complex(np.inf, 0)
    r = am.abft_group(X, Yf, "fp32")
    assert r["action"] == "rebuilt" and r["b"] == 2
    assert oracle.rel_l2(r["Y"], Y) < 1e-12
    Yf = Y.copy()
    Yf[1, 3] = np.nan
    Yf[3, 4] = np.inf
    assert am.abft_group(X, Yf, "fp32")["action"] == "uncorrectable"
    # two finite faults in different signals: ratio D1/D0 is not an index
    Yf = Y.copy()
    Yf[0, 1] += 1.0
    Yf[1, 9] += 1.0j
    r = am.abft_group(X, Yf, "fp32")
    assert r["action"] == "uncorrectable"
    # non-finite input: the group is not checked
    Xn = X.copy()
    Xn[0, 0] = np.nan
    assert am.abft_group(Xn, Y, "fp32")["action"] == "unchecked"


def test_flip_bit_helper():
    assert am.flip_bit(1.5 + 2j, 0, 31, "fp32") == complex(-1.5, 2)
    assert am.flip_bit(1.5 + 2j, 1, 63, "fp64") == complex(1.5, -2)
    assert am.flip_bit(1.0 + 0j, 0, 23, "fp32") == complex(0.5, 0)     # exponent LSB
    assert am.flip_bit(1.0 + 0j, 0, 52, "fp64") == complex(0.5, 0)
    assert am.flip_bit(1.0 + 0j, 0, 22, "fp32") == complex(1.5, 0)     # mantissa MSB


def test_gradient_closed_form_vs_finite_differences_and_torch():
    import torch
    rows, N = 3, 64
    x = synth.signals(rows, N, seed=4, dtype=np.complex128)
    w = synth.weights((rows, N), seed=5, dtype=np.float64)

    def loss(z):
        return float(np.sum(w * np.abs(oracle.fft(z)) ** 2))

    g = am.grad_sum_w_abs2(x, w)
    h = 1e-6
    fd = np.empty_like(x)
    for r in range(rows):
        for n in range(0, N, 7):
            e = np.zeros_like(x)
            e[r, n] = h
            dre = (loss(x + e) - loss(x - e)) / (2 * h)
            dim = (loss(x + 1j * e) - loss(x - 1j * e)) / (2 * h)
            fd[r, n] = dre + 1j * dim
    sel = (slice(None), slice(0, N, 7))
    assert oracle.rel_l2(g[sel], fd[sel]) < 1e-8
    xt = torch.tensor(x, requires_grad=True)
    lt = (torch.tensor(w) * torch.fft.fft(xt).abs() ** 2).sum()
    lt.backward()
    assert oracle.rel_l2(g, xt.grad.numpy()) < 1e-12


# --- per-transaction detection with delayed batched correction (Sec. 4.1) ---

def _group_with_faults(N, G, faults, seed):
    """Inputs, exact transforms (numpy.fft) and outputs with additive faults
    injected mid-transform (radix-2 DIT, stage and position per fault)."""
    X = synth.signals(G, N, seed=seed, dtype=np.complex128)
    Y = np.fft.fft(X)
    Yf = Y.copy()
    for b, stage, pos, eps in faults:
        Yf[b] = dit_radix2_with_fault(X[b], stage, pos, eps)
    return X, Y, Yf


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_per_transaction_clean_and_single_fault(precision):
    N, G = 64, 8
    X, Y, _ = _group_with_faults(N, G, [], seed=40)
    r = am.abft_group_per_transaction(X, Y, precision)
    assert r["faulty"] == [] and r["events"] == []
    assert np.array_equal(r["Y"], Y)
    lg = int(math.log2(N))
    for bstar in range(G):
        for stage in (0, lg // 2, lg):
            eps = 0.3 - 0.1j
            X, Y, Yf = _group_with_faults(N, G, [(bstar, stage, (3 * bstar + stage) % N, eps)], seed=41)
            r = am.abft_group_per_transaction(X, Yf, precision)
            # located exactly: the transaction whose own check failed
            assert r["faulty"] == [bstar]
            assert r["events"] == [(bstar, "corrected")]
            # Eq. 5 with the sums of the whole group: the corrected output is the DFT
            assert oracle.rel_l2(r["Y"], Y) < 1e-13


def test_per_transaction_two_faults_sequential():
    """Two faulty transactions in one group: the first is corrected when the
    second appears, from the right-side sums of the transactions before the
    second; the second at the end of the group.  Both end equal to the DFT,
    where the group-level check (one sum for the whole group) cannot tell
    them apart."""
    N, G = 128, 8
    for (b1, b2) in [(0, 7), (2, 3), (5, 6)]:
        X, Y, Yf = _group_with_faults(N, G, [(b1, 2, 9, 0.2 + 0.05j), (b2, 5, 77, -0.4j)], seed=42)
        r = am.abft_group_per_transaction(X, Yf, "fp64")
        assert r["faulty"] == [b1, b2]
        assert r["events"] == [(b1, "corrected"), (b2, "corrected")]
        assert oracle.rel_l2(r["Y"], Y) < 1e-13
        # one group sum holds both faults: whatever the group-level check
        # decides, it cannot restore both signals
        rg = am.abft_group(X, Yf, "fp64")
        assert rg["action"] == "uncorrectable" or oracle.rel_l2(rg["Y"], Y) > 1e-6


def test_per_transaction_non_finite_then_finite_fault():
    N, G = 64, 6
    X, Y, Yf = _group_with_faults(N, G, [(4, 3, 10, 0.5)], seed=43)
    Yf[1, 7] = complex(np.inf, 0.0)
    r = am.abft_group_per_transaction(X, Yf, "fp32")
    assert r["faulty"] == [1, 4]
    assert r["events"] == [(1, "rebuilt"), (4, "corrected")]
    assert oracle.rel_l2(r["Y"], Y) < 1e-12


def test_per_transaction_threshold_is_per_signal():
    """A fault in a weak signal of a strong group: above that signal's own
    threshold (so the per-transaction check finds it), below the threshold
    of the group's energy (so the group-level check cannot)."""
    N, G, kappa = 256, 8, 8.0
    X = synth.signals(G, N, seed=44, dtype=np.complex128)
    X[3] *= 1e-4
    Y = np.fft.fft(X)
    nu3 = float(np.sum(np.abs(X[3]) ** 2))
    nu = float(np.sum(np.abs(X) ** 2))
    tau3 = am.threshold(N, nu3, "fp32", kappa)
    tau_g = am.threshold(N, nu, "fp32", kappa)
    assert 20 * tau3 < tau_g
    Yf = Y.copy()
    Yf[3, 40] += 10 * tau3      # |e_k| = 1: D0 moves by exactly this much
    r = am.abft_group_per_transaction(X, Yf, "fp32", kappa=kappa)
    assert r["faulty"] == [3] and r["events"] == [(3, "corrected")]
    # the correction comes from sums over the whole group, 10^4 times the
    # weak signal: its rounding is u times that ratio
    assert oracle.rel_l2(r["Y"][3], Y[3]) < 1e-10
    assert am.abft_group(X, Yf, "fp32", kappa=kappa)["action"] == "clean"


def test_per_transaction_fp32_bit_flips_keep_each_signal_within_tolerance():
    """fp32 outputs as stored, every bit of one value per case, groups of
    G = 8: with each transaction checked against its own threshold, an
    undetected flip is at most tau_b / |e_k| = tau_b, a relative
    kappa u sqrt(log2 N) of its signal, independent of G -- so, unlike the
    group-level check, the group size is not bounded by the tolerance."""
    N, G, kappa, tol = 1024, 8, 8.0, 2e-6
    X = synth.signals(G, N, seed=45, dtype=np.complex64).astype(np.complex128)
    Y = np.fft.fft(X).astype(np.complex64).astype(np.complex128)
    worst_clean = 0.0
    for bit in range(31):
        for part in (0, 1):
            b, k = (bit + part) % G, (11 * bit + part) % N
            Yf = Y.copy()
            Yf[b, k] = am.flip_bit(complex(Y[b, k]), part, bit, "fp32")
            r = am.abft_group_per_transaction(X, Yf, "fp32", kappa=kappa)
            err = oracle.rel_l2(r["Y"][b], Y[b])
            assert err < tol, (bit, part, r["events"], err)
            if not r["faulty"]:
                assert abs(Yf[b, k] - Y[b, k]) <= r["tau"][b]
                worst_clean = max(worst_clean, err)
            else:
                assert r["faulty"] == [b] and r["events"][0][1] in ("corrected", "rebuilt")
    assert worst_clean < tol


# ---- thread-level check (Sec. 4.2, thread level) ----

@pytest.mark.parametrize("R", [2, 4, 8, 16])
def test_thread_left_vectors_closed_forms(R):
    """a_n is the geometric series (1 - w3^R) / (1 - w3 w_R^n); a1_n is the
    weighted series sum_k (k+1) z^k = (1 - (R+1) z^R + R z^(R+1)) / (1 - z)^2
    with z = w3 w_R^n."""
    a, a1 = am.thread_left_vectors(R)
    w3 = np.exp(-2j * np.pi / 3)
    n = np.arange(R)
    z = w3 * np.exp(-2j * np.pi * n / R)
    np.testing.assert_allclose(a, (1 - w3 ** R) / (1 - z), rtol=0, atol=1e-12)
    np.testing.assert_allclose(a1, (1 - (R + 1) * z ** R + R * z ** (R + 1)) / (1 - z) ** 2, rtol=0, atol=1e-11)


@pytest.mark.parametrize("R", [2, 4, 8, 16])
def test_thread_check_locates_and_corrects_every_output(R):
    rng = np.random.default_rng(R)
    v = rng.standard_normal(R) + 1j * rng.standard_normal(R)
    y0 = np.fft.fft(v)
    y, det, ks, mode = am.thread_dft_check(v, R)
    assert not det and ks is None
    for k in range(R):
        for delta in (0.3 * abs(y0[k]) + 0.1, -2.0j, 1e-3 * np.linalg.norm(v)):
            y, det, ks, mode = am.thread_dft_check(v, R, fault=(k, delta))
            assert det and ks == k and mode == "add", (k, delta)
            np.testing.assert_allclose(y, y0, rtol=0, atol=1e-12 * np.linalg.norm(v))
        # an exponent-sized error and a non-finite one are rebuilt
        for delta in (1e30, complex(np.inf, 0)):
            y, det, ks, mode = am.thread_dft_check(v, R, fault=(k, delta))
            assert det and ks == k and mode == "rebuild", (k, delta)
            np.testing.assert_allclose(y, y0, rtol=0, atol=1e-12 * np.linalg.norm(v))


def test_thread_check_no_false_alarm_in_fp32_rounding():
    """fp32 rounding of the transform and of the checksum products stays
    below the threshold (kappa = 8) over many random DFTs of every radix."""
    rng = np.random.default_rng(77)
    for R in (2, 4, 8, 16):
        a, a1 = am.thread_left_vectors(R)
        e = am.encoding_vector(R, 3)
        for _ in range(2000):
            v = (rng.uniform(-1, 1, R) + 1j * rng.uniform(-1, 1, R)).astype(np.complex64)
            p = np.complex64(np.sum(a.astype(np.complex64) * v))
            y = np.fft.fft(v.astype(np.complex128)).astype(np.complex64)
            q = np.complex64(np.sum(e.astype(np.complex64) * y))
            nu = float(np.vdot(v, v).real)
            tau = 8 * 2.0 ** -24 * np.sqrt(R * (np.log2(R) + 3)) * np.sqrt(nu)
            assert abs(complex(q) - complex(p)) <= tau, R


def test_location_fallback_finds_the_signal_when_the_code_is_noisy():
    """A fault above the threshold in a group of 32 whose outputs carry
    rounding-like noise (each signal's own checksum noise about 0.06 tau):
    the weighted sum D1 gathers the noise of every signal with weights up to
    32, so D1/D0 misses the index in most cases; the re-encoding fallback
    then still finds the faulty signal, and where the code does give an
    index the fallback is not consulted (brute force over seeds)."""
    G, N = 32, 256
    misses = 0
    for seed in range(40):
        rng = np.random.default_rng(1000 + seed)
        X = rng.uniform(-1, 1, (G, N)) + 1j * rng.uniform(-1, 1, (G, N))
        Y = np.fft.fft(X, axis=1)
        M = am.choose_M(N)
        tau = am.threshold(N, am.group_checksums(X, Y, M)["nu"], "fp32", 8.0)
        s = 0.35 * tau / np.sqrt(N * G)
        Y = Y + s * (rng.standard_normal((G, N)) + 1j * rng.standard_normal((G, N))) / np.sqrt(2)
        b0, k0 = int(rng.integers(0, G)), int(rng.integers(0, N))
        e = am.encoding_vector(N, M)
        Yf = Y.copy()
        Yf[b0, k0] += 2.0 * tau / abs(e[k0])
        plain = am.abft_group(X, Yf, "fp32", kappa=8.0)
        fb = am.abft_group(X, Yf, "fp32", kappa=8.0, fallback=True)
        assert plain["action"] != "clean", seed
        if plain["action"] == "uncorrectable":
            misses += 1
            assert fb["fallback"] and fb["b"] == b0 and fb["action"] in ("corrected", "rebuilt"), seed
        else:
            # the code gave an index (with this much noise not always the
            # right one): the fallback is not consulted
            assert fb["b"] == plain["b"] and not fb["fallback"], seed
    assert misses >= 10, misses
