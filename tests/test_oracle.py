"""Pins for the CPU oracle: the transform (TurboFFT Sec. 2.2).

Each check ties the oracle to something other than itself: hand-derived
values, closed forms, invariants, an independent library (numpy.fft), and the
O(N^2) definition on every small size.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dft_small.txt")


def _parse_vec(s):
    out = []
    for pair in s.strip().split(";"):
        re, im = pair.split(",")
        out.append(complex(float(re), float(im)))
    return np.array(out, dtype=np.complex128)


def _golden_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, N, d, xs, ys = [p.strip() for p in line.split("|")]
            cases.append((name, int(N), int(d), _parse_vec(xs), _parse_vec(ys)))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c[0])
def test_golden_hand_derived(case):
    name, N, d, x, y = case
    assert len(x) == N and len(y) == N
    for fn in (oracle.fft, oracle.dft):
        got = fn(x, dir=d)
        np.testing.assert_allclose(got, y, rtol=0, atol=4e-15)


SMALL_SIZES = sorted(set(list(range(1, 33)) + [1 << k for k in range(6, 11)] +
                         [3 << k for k in range(4, 9)] + [5 * 7, 9 * 11, 125]))


@pytest.mark.parametrize("N", SMALL_SIZES)
def test_fft_matches_definition_and_numpy(N):
    x = synth.signals(3, N, seed=N, dtype=np.complex128)
    for d in (-1, +1):
        y_fft = oracle.fft(x, dir=d, scale=1.0)
        y_dft = oracle.dft(x, dir=d, scale=1.0)
        scale = np.abs(y_dft).max() + 1.0
        assert np.abs(y_fft - y_dft).max() <= 64 * 2.0 ** -53 * scale * max(1, N)
        ref = np.fft.fft(x) if d == -1 else np.fft.ifft(x) * N
        assert np.abs(y_fft - ref).max() <= 64 * 2.0 ** -53 * scale * max(1.0, math.log2(N) + 1)


def test_twiddle_exact_points_and_accuracy():
    # exact symmetry points of the unit circle
    assert oracle.twiddle(4, 1, -1) == complex(0.0, -1.0)
    assert oracle.twiddle(4, 2, -1) == complex(-1.0, 0.0)
    assert oracle.twiddle(4, 3, +1) == complex(0.0, -1.0)
    assert oracle.twiddle(8, 0, -1) == 1.0
    assert oracle.twiddle(2, 1, +1) == complex(-1.0, 0.0)
    # m is reduced modulo N exactly, including huge and negative exponents
    assert oracle.twiddle(12, 12 * 10 ** 12 + 5, -1) == oracle.twiddle(12, 5, -1)
    assert oracle.twiddle(12, -7, -1) == oracle.twiddle(12, 5, -1)
    rng = np.random.default_rng(1)
    for N in (3, 7, 64, 96, 1 << 20, 3 << 16):
        for m in rng.integers(0, N, size=50):
            w = oracle.twiddle(N, int(m), -1)
            ref = complex(math.cos(2 * math.pi * (m / N)), -math.sin(2 * math.pi * (m / N)))
            # the float reference angle 2*pi*(m/N) itself carries ~1 ulp error
            assert abs(w - ref) <= 1e-15
            assert abs(abs(w) - 1.0) <= 4e-16
    # points with known surds: w_3 = -1/2 - i sqrt(3)/2, w_12 = sqrt(3)/2 - i/2
    s3 = math.sqrt(3.0) / 2
    assert abs(oracle.twiddle(3, 1, -1) - complex(-0.5, -s3)) <= 1.2e-16
    assert abs(oracle.twiddle(12, 1, -1) - complex(s3, -0.5)) <= 1.2e-16
    assert abs(oracle.twiddle(8, 3, -1) - complex(-math.sqrt(0.5), -math.sqrt(0.5))) <= 1.2e-16


@pytest.mark.parametrize("N", [8, 64, 96, 1024, 3072])
def test_closed_forms(N):
    n = np.arange(N)
    # impulse at m: y_k = w_N^{k m}
    for m in (0, 1, N // 3, N - 1):
        x = np.zeros(N, complex)
        x[m] = 1
        ref = np.exp(-2j * np.pi * ((n * m) % N) / N)
        np.testing.assert_allclose(oracle.fft(x), ref, rtol=0, atol=1e-13)
    # pure tone at f: y = N delta_{k f}
    for f in (0, 1, N // 2 + 1):
        x = np.exp(2j * np.pi * ((f * n) % N) / N)
        ref = np.zeros(N, complex)
        ref[f] = N
        np.testing.assert_allclose(oracle.fft(x), ref, rtol=0, atol=1e-11 * N)
    # constant: y = N delta_{k 0}
    ref = np.zeros(N, complex)
    ref[0] = N * (0.5 - 0.25j)
    np.testing.assert_allclose(oracle.fft(np.full(N, 0.5 - 0.25j)), ref, rtol=0, atol=1e-12 * N)


@pytest.mark.parametrize("N", [64, 96, 4096, 3 << 10])
def test_invariants(N):
    x = synth.signals(4, N, seed=7, dtype=np.complex128)
    z = synth.signals(4, N, seed=8, dtype=np.complex128)
    y = oracle.fft(x)
    # Parseval: sum |y|^2 = N sum |x|^2
    np.testing.assert_allclose((np.abs(y) ** 2).sum(1), N * (np.abs(x) ** 2).sum(1), rtol=1e-12)
    # linearity
    a, b = 0.3 - 1.1j, -2.0 + 0.5j
    np.testing.assert_allclose(oracle.fft(a * x + b * z), a * y + b * oracle.fft(z),
                               rtol=0, atol=1e-12 * N)
    # inverse round trip (dir +1 scales by 1/N)
    np.testing.assert_allclose(oracle.fft(y, dir=+1), x, rtol=0, atol=1e-14 * math.log2(N))
    # Hermitian symmetry for real input: y_{N-k} = conj(y_k)
    yr = oracle.fft(x.real)
    np.testing.assert_allclose(yr[:, (-np.arange(N)) % N], np.conj(yr), rtol=0, atol=1e-12 * N)
    # time shift by s multiplies by w_N^{ks}
    s = 5
    ys = oracle.fft(np.roll(x, s, axis=1))
    k = np.arange(N)
    np.testing.assert_allclose(ys, y * np.exp(-2j * np.pi * ((k * s) % N) / N),
                               rtol=0, atol=1e-12 * N)


def test_dft_bins_and_threads():
    N = 3 << 12
    x = synth.signals(5, N, seed=3, dtype=np.complex128)
    y1 = oracle.fft(x, threads=1)
    y4 = oracle.fft(x, threads=4)
    assert np.array_equal(y1, y4)
    ks = [0, 1, 17, N // 2, N - 1]
    np.testing.assert_allclose(oracle.dft_bins(x[2], ks), y1[2, ks], rtol=0, atol=1e-9)


def test_complex64_input_is_upcast_exactly():
    x = synth.signals(2, 256, seed=11, dtype=np.complex64)
    y = oracle.fft(x)
    y64 = oracle.fft(x.astype(np.complex128))
    assert np.array_equal(y, y64)


def test_rel_l2():
    r = np.array([3 + 4j, 0])
    assert oracle.rel_l2(r, r) == 0.0
    assert abs(oracle.rel_l2(r + np.array([0.5, 0]), r) - 0.1) < 1e-15
