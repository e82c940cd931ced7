"""CPU reference model of two-side ABFT with location encoding -- TEST INFRASTRUCTURE ONLY.

Follows TurboFFT Sec. 2.2 (checksum identity (e^T W) x = e^T (W x), Eq. 1-2,
the encoding-vector discussion and the threshold test), Sec. 4.1 (two-side
checksum X^c = [X, Xe], Y^c = W^c X^c, Eq. 4-5; location encoding with the
weights e_3 = (1, 2, ...); delayed batched correction) and Sec. 4.3
(multi-transaction groups, location weight = the signal's index in the group).
All arithmetic here is fp64 numpy plus the oracle FFT of this package.

Readings taken where the paper is silent:
  * encoding vector e_k = w_M^k, w_M = exp(-2 pi i / M), M = 3 (Wang's vector),
    switched to M = 5 when 3 | N (then w_3 makes e^T W vanish almost everywhere);
  * left vector a = e^T W = W e (W is symmetric), closed form
    a_n = (1 - w_M^N) / (1 - w_M w_N^n);
  * location weights are group-local, 1-based: w_b = b + 1;
  * absolute threshold tau = kappa * u * sqrt(N log2 N) * sqrt(nu) with nu the
    group's input energy, instead of the relative test, which fails when the
    checksum is near zero;
  * an output value that is not finite or exceeds the magnitude cap H marks its
    signal as corrupted directly (exponent flips);
  * correction adds c = W(Xe) - Ye to the located signal when c is small
    (max |c| <= rms output norm of one signal), otherwise rebuilds the signal
    as W(Xe) - sum of the other outputs;
  * two detection granularities: once per group with location encoding
    (abft_group), or per transaction with its own threshold and delayed
    correction from the right-side sums so far (abft_group_per_transaction);
  * location fallback (abft_group, fallback=True): when D1/D0 is not an
    index, each signal is re-encoded on its own and the largest |d_b| taken.

Also the thread-level check of one radix-R DFT (thread_dft_check).

Parity unpinned: the threshold constant kappa (no worked value in the paper);
the tests pin every decision for faults well away from the threshold.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as _oracle_fft

UNIT_ROUNDOFF = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}
MAG_CAP = {"fp32": 2.0 ** 64, "fp64": 2.0 ** 512}


def choose_M(N: int) -> int:
    """Period of the encoding vector: 3, or 5 when 3 divides N."""
    return 5 if N % 3 == 0 else 3


def encoding_vector(N: int, M: int, sign: int = -1) -> np.ndarray:
    """e_k = exp(sign 2 pi i k / M), k = 0..N-1 (Wang-type vector)."""
    k = np.arange(N) % M
    return np.exp(sign * 2j * np.pi * k / M)


def left_vector(N: int, M: int, dir: int = -1) -> np.ndarray:
    """a = e^T W_dir computed as the transform of e (W_dir is symmetric)."""
    e = encoding_vector(N, M)
    return _oracle_fft(e, dir=dir, scale=1.0)


def left_vector_closed_form(N: int, M: int, dir: int = -1) -> np.ndarray:
    """a_n = (1 - w_M^N) / (1 - w_M w_N^{dir n}) -- geometric series in k."""
    wm = np.exp(-2j * np.pi / M)
    n = np.arange(N)
    wn = np.exp(dir * 2j * np.pi * n / N)
    return (1 - wm ** N) / (1 - wm * wn)


def threshold(N: int, nu: float, precision: str, kappa: float) -> float:
    """tau = kappa * u * sqrt(N log2 N) * sqrt(nu)."""
    u = UNIT_ROUNDOFF[precision]
    lg = math.log2(N) if N > 1 else 1.0
    return kappa * u * math.sqrt(N * lg) * math.sqrt(max(nu, 0.0))


def flip_bit(value: complex, part: int, bit: int, precision: str) -> complex:
    """Flip one bit of the real (part=0) or imaginary (part=1) component,
    as stored in binary32 or binary64 (Sec. 5.3 injection protocol)."""
    if precision == "fp32":
        arr = np.array([value.real, value.imag], dtype=np.float32)
        u = arr.view(np.uint32)
        u[part] ^= np.uint32(1 << bit)
    else:
        arr = np.array([value.real, value.imag], dtype=np.float64)
        u = arr.view(np.uint64)
        u[part] ^= np.uint64(1 << bit)
    return complex(float(arr[0]), float(arr[1]))


def group_checksums(X: np.ndarray, Y: np.ndarray, M: int, dir: int = -1):
    """Left/right, plain/location-weighted checksums of one group (Eq. 4-5).

    X, Y: [G, N].  Returns dict with s_in, l_in, s_out, l_out (complex),
    x_s = X e_c, y_s = Y e_c (the right-side sums, e_c = ones), nu = sum |x|^2.
    """
    G, N = X.shape
    a = left_vector(N, M, dir)
    e = encoding_vector(N, M)
    w = np.arange(1, G + 1, dtype=np.float64)
    with np.errstate(all="ignore"):
        p = X @ a            # a^T x_b per signal
        q = Y @ e            # e^T y_b per signal
        return {
            "s_in": p.sum(), "l_in": (w * p).sum(),
            "s_out": q.sum(), "l_out": (w * q).sum(),
            "x_s": X.sum(axis=0), "y_s": Y.sum(axis=0),
            "nu": float(np.sum(np.abs(X) ** 2)),
        }


def abft_group(X, Yp, precision: str = "fp32", kappa: float = 32.0, dir: int = -1,
               M: int | None = None, rho: float = 0.25, fallback: bool = False):
    """Detect, locate and correct one group (Sec. 4.1-4.3).

    X  : [G, N] inputs of the group's signals.
    Yp : [G, N] unscaled transforms as produced, possibly with one fault.
    fallback: when D1/D0 is not an index (an error just above the threshold,
    where the rounding of the weighted sum dominates), re-encode every
    signal of the group on its own, d_b = e^T y_b - a^T x_b, and take the one
    with the largest |d_b| (the inputs being intact) instead of giving up.
    Returns a dict: action in {"clean", "corrected", "rebuilt", "uncorrectable",
    "unchecked"}, located index b (or None), corrected outputs Y, D0, D1, tau,
    and "fallback" (the location came from the re-encoding).
    """
    X = np.asarray(X, dtype=np.complex128)
    Y = np.array(Yp, dtype=np.complex128, copy=True)
    G, N = X.shape
    if M is None:
        M = choose_M(N)
    cs = group_checksums(X, Y, M, dir)
    nu = cs["nu"]
    res = {"action": "clean", "b": None, "Y": Y, "tau": None, "D0": None, "D1": None, "fallback": False}
    if not math.isfinite(nu):
        res["action"] = "unchecked"      # non-finite input: nothing to protect
        return res
    tau = threshold(N, nu, precision, kappa)
    cap = MAG_CAP[precision]
    with np.errstate(all="ignore"):
        D0 = cs["s_out"] - cs["s_in"]
        D1 = cs["l_out"] - cs["l_in"]
        bad = ~(np.abs(Y.real) <= cap) | ~(np.abs(Y.imag) <= cap)
    res.update(tau=tau, D0=D0, D1=D1)
    nf = sorted(set(np.nonzero(bad.any(axis=1))[0].tolist()))
    if len(nf) > 1:
        res["action"] = "uncorrectable"
        return res
    if len(nf) == 1:
        b = nf[0]
    elif not (abs(D0) <= tau):
        r = D1 / D0
        b = int(round(r.real)) - 1
        if not (0 <= b < G and abs(r - (b + 1)) <= rho):
            if not fallback:
                res["action"] = "uncorrectable"
                return res
            a = left_vector(N, M, dir)
            e = encoding_vector(N, M)
            d = Y @ e - X @ a
            b = int(np.argmax(np.abs(d)))
            res["fallback"] = True
    else:
        return res
    res["b"] = b
    # Right-side correction: c = W (X e_c) - Y' e_c = -(fault) under SEU (Eq. 5).
    Wxs = _oracle_fft(cs["x_s"], dir=dir, scale=1.0)
    with np.errstate(all="ignore"):
        c = Wxs - cs["y_s"]
        y_rms = math.sqrt(N * nu / G)
        small = bool(np.all(np.isfinite(c))) and float(np.max(np.abs(c))) <= y_rms and not nf
    e = encoding_vector(N, M)
    if small:
        Y[b] = Y[b] + c
        ok = abs(np.dot(e, c) + D0) <= tau
        res["action"] = "corrected" if ok else "uncorrectable"
    else:
        others = np.delete(Y, b, axis=0).sum(axis=0)
        Y[b] = Wxs - others
        ok = bool(np.all(np.abs(Y[b].real) <= cap) and np.all(np.abs(Y[b].imag) <= cap))
        res["action"] = "rebuilt" if ok else "uncorrectable"
    res["Y"] = Y
    return res


def abft_group_per_transaction(X, Yp, precision: str = "fp32", kappa: float = 32.0, dir: int = -1,
                               M: int | None = None):
    """Per-transaction detection with delayed batched correction (Sec. 4.1,
    "Delayed Batched Correction"; Sec. 4.3 multi-transaction groups).

    Each transaction b checks its own left-side checksum, p_b = (e^T W) x_b
    against q_b = e^T y_b, with its own threshold tau_b (its input energy
    nu_b).  A faulty transaction is noted and processing continues; the
    right-side sums x_s = sum x_b, y_s = sum y_b are added at the END of each
    transaction, after its check, so a second fault cannot contaminate sums
    that already hold one.  The noted transaction is corrected when the next
    fault appears or the group ends, from the sums accumulated so far:
    c = W x_s - y_s (= minus its fault, Eq. 5), y_b += c and y_s += c, or,
    when c is not finite or larger than one signal's rms output norm, a
    rebuild y_b = W x_s - (sum of the other outputs in the sums).  An
    additive correction is accepted when |e^T c + D0_b| stays within the
    threshold of the summed transactions' energy (the rounding of c comes
    from all of them; in exact arithmetic e^T c = -D0_b).

    X, Yp: [G, N] inputs and unscaled outputs as produced.  Returns a dict:
    "Y" the repaired outputs, "events" a list of (b, action) with action in
    {"corrected", "rebuilt", "uncorrectable"} in the order they were taken,
    "faulty" the transactions found faulty, "tau" the per-transaction
    thresholds and "D0" the per-transaction differences q_b - p_b.
    """
    X = np.asarray(X, dtype=np.complex128)
    Y = np.array(Yp, dtype=np.complex128, copy=True)
    G, N = X.shape
    if M is None:
        M = choose_M(N)
    a = left_vector(N, M, dir)
    e = encoding_vector(N, M)
    cap = MAG_CAP[precision]
    x_s = np.zeros(N, np.complex128)
    n_in = 0                        # transactions added to the sums
    nu_s = 0.0
    taus, d0s, faulty, events = [], [], [], []
    pending = None                  # (b, D0_b, tau_b, non-finite)

    def correct(pend):
        b, d, tau, nonfinite = pend
        Wxs = _oracle_fft(x_s, dir=dir, scale=1.0)
        others = [j for j in range(n_in) if j != b]
        with np.errstate(all="ignore"):
            y_others = Y[others].sum(axis=0) if others else np.zeros(N, np.complex128)
            c = Wxs - (y_others + Y[b])
            y_rms = math.sqrt(N * nu_s / max(n_in, 1))
            small = (not nonfinite) and bool(np.all(np.isfinite(c))) and float(np.max(np.abs(c))) <= y_rms
        if small:
            Y[b] = Y[b] + c
            # c carries the rounding of every signal in the sums, so the
            # check that it explains the discrepancy uses their energy
            tau_v = threshold(N, nu_s, precision, kappa)
            ok = abs(np.dot(e, c) + d) <= tau_v
            events.append((b, "corrected" if ok else "uncorrectable"))
        else:
            Y[b] = Wxs - y_others
            ok = bool(np.all(np.abs(Y[b].real) <= cap) and np.all(np.abs(Y[b].imag) <= cap))
            events.append((b, "rebuilt" if ok else "uncorrectable"))

    for b in range(G):
        nu_b = float(np.sum(np.abs(X[b]) ** 2))
        tau_b = threshold(N, nu_b, precision, kappa) if math.isfinite(nu_b) else math.inf
        with np.errstate(all="ignore"):
            d = np.dot(e, Y[b]) - np.dot(a, X[b])
            nonfinite = bool(np.any(~(np.abs(Y[b].real) <= cap) | ~(np.abs(Y[b].imag) <= cap)))
        taus.append(tau_b)
        d0s.append(d)
        checked = math.isfinite(nu_b)
        if checked and (nonfinite or not (abs(d) <= tau_b)):
            faulty.append(b)
            if pending is not None:
                correct(pending)        # sums over the transactions before b
            pending = (b, d, tau_b, nonfinite)
        # right-side sums at the end of the transaction
        x_s += X[b]
        nu_s += nu_b if checked else 0.0
        n_in += 1
    if pending is not None:
        correct(pending)
    return {"Y": Y, "events": events, "faulty": faulty, "tau": taus, "D0": d0s}


def grad_sum_w_abs2(x, w) -> np.ndarray:
    """Gradient of L = sum w * |FFT(x)|^2 w.r.t. complex x, PyTorch convention
    (dL/dRe + i dL/dIm): 2 * conj(W)^T (w * y) = 2 * (unscaled inverse DFT)(w * y)."""
    y = _oracle_fft(x, dir=-1, scale=1.0)
    return _oracle_fft(2.0 * np.asarray(w) * y, dir=+1, scale=1.0)


# ---------------------------------------------------------------------------
# Thread-level two-side ABFT (Sec. 4.2, thread level): one radix-R DFT held
# by one lane is checked, located and corrected on its own.
# ---------------------------------------------------------------------------

def thread_left_vectors(R: int) -> tuple[np.ndarray, np.ndarray]:
    """(a, a1) with a = e^T W_R and a1 = e1^T W_R, e_k = w_3^k and
    e1_k = (k + 1) w_3^k (the location weights), W_R the forward R-point DFT
    matrix; computed as the transforms of e and e1 (W_R is symmetric)."""
    e = encoding_vector(R, 3)
    e1 = e * (np.arange(R) + 1)
    return _oracle_fft(e, dir=-1, scale=1.0), _oracle_fft(e1, dir=-1, scale=1.0)


def thread_dft_check(v, R: int, precision: str = "fp32", kappa: float = 8.0, fault=None):
    """Run one radix-R DFT of v under the thread-level check.

    Steps in the order of the scheme: encode the inputs (p = a^T v,
    p1 = a1^T v, nu = |v|^2); transform (y = W_R v); optionally add a fault
    (k, delta) to output k; encode the outputs (q = e^T y, q1 = e1^T y);
    detect with |q - p| > tau, tau = kappa u sqrt(R (log2 R + 3)) sqrt(nu);
    locate k* = round(Re((q1 - p1) / (q - p))) - 1; correct y_{k*} -= (q - p)
    / e_{k*} when |q - p| <= 32 sqrt(nu), else rebuild the largest output
    from the left checksum, e_{k*} y_{k*} = p - sum_{k != k*} e_k y_k.
    Returns (y, detected, k_star, mode) with mode None, "add" or "rebuild"."""
    v = np.asarray(v, dtype=np.complex128)
    a, a1 = thread_left_vectors(R)
    e = encoding_vector(R, 3)
    e1 = e * (np.arange(R) + 1)
    p, p1 = a @ v, a1 @ v
    nu = float(np.vdot(v, v).real)
    y = _oracle_fft(v, dir=-1, scale=1.0)
    if fault is not None:
        k, delta = fault
        y = y.copy()
        y[k] += delta
    with np.errstate(invalid="ignore", over="ignore"):   # a non-finite fault
        q, q1 = e @ y, e1 @ y
    d = q - p
    tau = kappa * UNIT_ROUNDOFF[precision] * math.sqrt(R * (math.log2(R) + 3)) * math.sqrt(nu)
    if not (abs(d) <= tau):
        if np.isfinite(d) and abs(d) <= 32 * math.sqrt(nu):
            ks = int(round(((q1 - p1) / d).real)) - 1
            if 0 <= ks < R:
                y = y.copy()
                y[ks] -= d / e[ks]
                return y, True, ks, "add"
        with np.errstate(invalid="ignore"):
            mags = np.where(np.isfinite(np.abs(y)), np.abs(y.real) + np.abs(y.imag), np.inf)
        ks = int(np.argmax(mags))
        y = y.copy()
        others = sum(e[m] * y[m] for m in range(R) if m != ks)
        y[ks] = (p - others) / e[ks]
        return y, True, ks, "rebuild"
    return y, False, None, None
