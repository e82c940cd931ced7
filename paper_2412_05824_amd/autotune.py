"""Offline autotuner: measure every built configuration of each length and
write the fastest into a JSON tuning table that the library loads
(tfft_load_tuning).

Per (precision, N) it sweeps, with ABFT correction on:
  * the route: single pass (when built) or each column/row split n1 x N/n1
    (the multi-pass decomposition of Sec. 3.1), over the compiled plan
    variants (tile width, elements per lane) of each pass;
  * the detection granularity: once per group of T transactions with the
    location code (Sec. 4.3), or per transaction with delayed batched
    correction (Sec. 4.1), and T, the transactions per group, limited by
    the accuracy bounds below;
  * for two-pass routes, the chunk of signals whose intermediate lives in
    the workspace;
then, without ABFT, T and the chunk again on the same route (a shared plan
keeps outputs bit-identical whether ABFT is on or off).
With --ragged-only it tunes the ragged batch's schedule instead (elements
per work item, register budget of the persistent ABFT kernel) on a seeded
batch drawn from the ragged menu, and stores it under "ragged".
Each candidate runs on a 1 GiB seeded batch; it must count no detection on
fault-free data and agree with the default configuration's output to
within twice the precision's tolerance (two correct transforms differ by at
most the sum of their errors).

Accuracy bounds on T.  Checked once per group, a flip just below the
detection threshold changes one signal by about kappa * u * sqrt(T * s) of its
norm, s the rounding steps per element the threshold counts (log2 Ns, plus 3
in a pass with an inter-pass twiddle; the largest over the route's passes),
which must stay under the acceptance tolerance (2e-6 fp32, 1e-13 fp64), so
T <= (tol / (kappa * u))^2 / s.
Checked per transaction, each signal has its own threshold; T then only sets
how many signals share the right-side sums of a correction, whose rounding
(about u * sqrt(T * s) of one signal's norm) stays far below the
tolerance up to T = 16, the most a plan keeps; the library reduces a larger
T to what the plan keeps, and the tuner skips such duplicates.

    python -m paper_2412_05824_amd.autotune --out paper_2412_05824_amd/tuning/mi355x.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

TOL = {"fp32": 2e-6, "fp64": 1e-13}
UNIT = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}
KAPPA = {"fp32": 8.0, "fp64": 16.0}
T_CHOICES = (1, 2, 4, 8, 16)
GRANS = {"fp32": (1, 0), "fp64": (0, 1)}   # per transaction, per group
CHUNKS_MIB = (16, 32, 64, 128, 256, 512)


def steps(N: int, n1: int, n2: int = 0) -> float:
    """Rounding steps per element the threshold counts, the largest over the
    passes of the route (single pass: n1 = 1; two passes: n1, N / n1; three:
    n1, n2, N / (n1 n2)); passes after the first carry an inter-pass twiddle."""
    if n1 <= 1:
        return math.log2(N)
    rest = [n2, N // (n1 * n2)] if n2 else [N // n1]
    return max([math.log2(n1)] + [math.log2(m) + 3 for m in rest])


def max_T(prec: str, s: float, kappa: float) -> int:
    lim = (TOL[prec] / (kappa * UNIT[prec])) ** 2 / max(1.0, s)
    return max(1, int(lim))


def _time(fn, torch, reps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(precisions, logs, modes=(2, 0), reps=5, warmup=2, total_bytes=1 << 30, log=print):
    import numpy as np
    import torch

    import paper_2412_05824_amd as tf

    dev = torch.device("cuda:0")
    entries = []
    for prec in precisions:
        dtype = torch.complex64 if prec == "fp32" else torch.complex128
        npdt = np.complex64 if prec == "fp32" else np.complex128
        esize = 8 if prec == "fp32" else 16
        total = total_bytes // esize
        # re, im i.i.d. U[-1, 1) from a seeded device generator
        g = torch.Generator(device=dev)
        g.manual_seed(4000)
        rdt = torch.float32 if prec == "fp32" else torch.float64
        x = (torch.rand(total, 2, dtype=rdt, device=dev, generator=g) * 2 - 1).view(dtype).view(-1)
        y = torch.empty_like(x)
        ref = torch.empty_like(x)
        counts = tf.new_counts(dev)
        for lg in logs:
            N = 1 << lg
            if not tf.supported(N, dtype):
                continue
            xv, yv, rv = x.view(-1, N), y.view(-1, N), ref.view(-1, N)
            T0, k0 = tf.get_tuning(N, dtype)
            gran0 = tf.route_info(N, dtype, 2)["gran"]
            tf.set_route(N, dtype, 0)
            tf.fft_c2c(xv, ft_mode=tf.FT_OFF, out=rv)
            torch.cuda.synchronize()
            ref_norm = torch.linalg.vector_norm(rv).item()
            best_code = None
            for ft in modes:
                best = None
                # every mode runs the plan chosen for the first (correcting)
                # mode, so switching ABFT on or off never changes an output
                # bit; the other modes tune only T and the chunk
                codes = tf.routes(N, dtype, ft) if best_code is None else [best_code]
                for code in codes:
                    n1, va, vb = tf.route_parts(code)
                    n2 = tf.route_n2(code)
                    s_route = steps(N, n1, n2)
                    chunks = [None] if n1 == 1 else [c << 20 for c in CHUNKS_MIB]
                    cands = []
                    for gran in (GRANS[prec] if ft else (0,)):
                        # without ABFT, T only sets the signals per workgroup
                        tmax = 4 if not ft else (16 if gran else max_T(prec, s_route, KAPPA[prec]))
                        seen = set()
                        for T in [t for t in T_CHOICES if t <= tmax]:
                            tf.set_route(N, dtype, code)
                            tf.set_granularity(N, dtype, gran)
                            tf.set_tuning(N, dtype, T, KAPPA[prec])
                            teff = tf.route_info(N, dtype, ft)["T"]
                            if teff in seen:
                                continue   # reduced to a T already measured
                            seen.add(teff)
                            cands.append((gran, T))
                    for gran, T in cands:
                        for chunk in chunks:
                            tf.set_route(N, dtype, code)
                            tf.set_granularity(N, dtype, gran)
                            tf.set_tuning(N, dtype, T, KAPPA[prec])
                            if chunk:
                                tf.set_chunk(N, dtype, chunk)
                            counts.zero_()
                            ms = _time(lambda: tf.fft_c2c(xv, ft_mode=ft, out=yv, counts=counts),
                                       torch, reps, warmup)
                            det = tf.counts_dict(counts)["detected"]
                            err = torch.linalg.vector_norm(yv - rv).item() / ref_norm
                            ok = det == 0 and err <= 2 * TOL[prec]
                            gbs = 2 * total * esize / (ms * 1e-3) / 1e9
                            log(f"{prec} N={N} ft={ft} n1={n1} n2={n2} v={va}/{vb} gran={gran} T={T} chunk={chunk} {ms:.4f} ms "
                                f"{gbs:.1f} GB/s err={err:.2e} det={det}{'' if ok else ' REJECTED'}")
                            if ok and (best is None or ms < best["ms"]):
                                best = {"precision": prec, "N": N, "ft_mode": ft, "split_n1": n1,
                                        "split_n2": n2,
                                        "variant_a": va, "variant_b": vb, "T": T, "gran": gran,
                                        "kappa": KAPPA[prec],
                                        "ms": round(ms, 5), "gbs": round(gbs, 1)}
                                if chunk:
                                    best["chunk_bytes"] = chunk
                if best:
                    entries.append(best)
                    log(f"best {prec} N={N} ft={ft}: {best}")
                    if best_code is None:
                        best_code = tf.route_code(best["split_n1"], best["variant_a"], best["variant_b"],
                                                  best["split_n2"])
                # back to the defaults before the next mode / length
                tf.set_route(N, dtype, 0)
                tf.set_tuning(N, dtype, T0, k0)
                tf.set_granularity(N, dtype, gran0)
                tf.set_chunk(N, dtype, 128 << 20)
        del x, y, ref
        torch.cuda.empty_cache()
    return entries


RAGGED_ITEMS = (8192, 16384, 32768, 65536)
RAGGED_WAVES = (3, 0)


def tune_ragged(signals=10000, seed=5, reps=5, log=print):
    """The ragged batch's schedule: elements per work item and the ABFT
    kernels' register budget, on a seeded batch of `signals` lengths drawn
    uniformly from the ragged menu (2^k and 3 * 2^k, 6 <= k <= 16), forward,
    ABFT correct, one persistent launch; the fastest setting that counts no
    detection and matches the per-size launches bit for bit."""
    import numpy as np
    import torch

    import paper_2412_05824_amd as tf

    dev = torch.device("cuda:0")
    menu = [n for k in range(6, 17) for n in (1 << k, 3 << k) if tf.ragged_supported(n)]
    rng = np.random.default_rng(seed)
    sizes = [int(n) for n in rng.choice(menu, size=signals)]
    total = int(sum(sizes))
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    x = (torch.rand(total, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(-1)
    y = torch.empty_like(x)
    ref = torch.empty_like(x)
    counts = tf.new_counts(dev)
    best = None
    first = True
    for waves in RAGGED_WAVES:
        for item in RAGGED_ITEMS:
            tf.ragged_set_schedule(0, item, waves)
            plan = tf.RaggedPlan(sizes, device=dev)
            try:
                if first:
                    plan(x, out=ref, ft_mode=tf.FT_CORRECT, counts=counts, mode="per_size")
                    first = False
                run = lambda: plan(x, out=y, ft_mode=tf.FT_CORRECT, counts=counts, mode="persistent")
                counts.zero_()
                ms = _time(run, torch, reps, 2)
                ok = tf.counts_dict(counts)["detected"] == 0 and bool(torch.equal(y, ref))
            finally:
                plan.close()
            log(f"ragged item={item} waves={waves}: {ms:.4f} ms{'' if ok else ' REJECTED'}")
            if ok and (best is None or ms < best["ms"]):
                best = {"item_elems": item, "waves": waves, "ms": round(ms, 5),
                        "workload": f"{signals} signals, ragged menu, seed {seed}, {total} elements"}
    tf.ragged_set_schedule(0, 32768, 3)
    del x, y, ref
    torch.cuda.empty_cache()
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--precision", default="fp32,fp64")
    ap.add_argument("--sizes", default="6-22", help="log2 N range lo-hi or comma list")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--ragged-only", action="store_true",
                    help="tune only the ragged schedule and store it in the existing table --out")
    args = ap.parse_args(argv)
    if args.ragged_only:
        with open(args.out) as f:
            doc = json.load(f)
        best = tune_ragged(reps=args.reps, log=lambda s: print(s, flush=True))
        if best:
            doc["ragged"] = best
        with open(args.out, "w") as f:
            json.dump(doc, f, indent=1)
        import paper_2412_05824_amd as tf
        print(f"wrote {args.out}: ragged {best}, {tf.load_tuning(args.out)} entries", flush=True)
        return 0
    if "-" in args.sizes:
        lo, hi = (int(v) for v in args.sizes.split("-"))
        logs = list(range(lo, hi + 1))
    else:
        logs = [int(v) for v in args.sizes.split(",")]
    import torch
    t0 = time.time()
    entries = tune(args.precision.split(","), logs, reps=args.reps,
                   log=lambda s: print(s, flush=True))
    doc = {"format": "tfft-tuning-1",
           "device": torch.cuda.get_device_name(0),
           "workload": "1 GiB seeded batch per length, forward, ABFT correct and off",
           "seconds": round(time.time() - t0, 1),
           "entries": entries}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    # the library must accept what was written
    import paper_2412_05824_amd as tf
    n = tf.load_tuning(args.out)
    print(f"wrote {args.out}: {n} entries", flush=True)


if __name__ == "__main__":
    sys.exit(main())
