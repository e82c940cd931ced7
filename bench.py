"""Benchmark: batched fp32 C2C FFT with fused two-side ABFT on one MI355X.

Workload (the headline sweep): complex64 forward transforms, N = 2^6 .. 2^22,
batch = 2^27 / N (1 GiB per buffer), inputs U[-1, 1) re/im, ABFT on
(TFFT_FT_CORRECT).  One step = one launch per N over its whole 1 GiB batch,
inputs resident in HBM.  value = algorithmic bytes (read x + write y,
2 * N * batch * 8 per launch) summed over the sweep / step time, in GB/s.

Printed as ONE JSON line, with:
  * sweep: per N, effective GB/s with ABFT off, on, and on under injection
    (one seeded single-bit flip per 100 launches), ABFT overhead and counts;
  * roofline: the kernel that takes most of the step, HBM-bound, achieved
    GB/s from HIP events on the launch stream against 8 TB/s (the warmup
    steps time every launch and pick the kernel; the timed steps bracket
    only that kernel's launches, so the step time carries few events);
  * kernels: every kernel's launches, time and bytes (warmup steps);
  * cpu_baseline: the fp64 CPU oracle on a bounded sample of the same sweep;
  * fp64_sweep: complex128 forward and inverse, N = 2^6..2^20, batch 2^26/N,
    standard-normal inputs, ABFT off and correct, seeded single-bit flips;
  * three_pass: complex64 forward transforms of N = 2^23..2^29 as three
    launches, ABFT off and correct, per-pass kernel times, one seeded flip
    in each pass;
  * autograd: loss = sum(w * |FFT(x)|^2) on x complex64 [16384, 4096], one
    forward + backward (ABFT-protected adjoint) per step;
  * ragged: 10,000 signals with lengths drawn uniformly from {2^k, 3*2^k :
    6 <= k <= 16} (seeded), ABFT on, as one persistent launch replayed from a
    captured graph against one launch per length and pass (eager and
    captured), same kernel bodies.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TOTAL_ELEMS = 1 << 27          # 1 GiB of complex64 per buffer


def streaming_reference(torch, stream, x, y, reps=20):
    """GB/s (read + write bytes) of torch's own 1 GiB device copy and in-place
    complex scale on the benchmark buffers: what a plain streaming kernel
    reaches here, beside the 8 TB/s peak."""
    nbytes = 2 * x.numel() * x.element_size()

    def rate(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            best = ms if best is None else min(best, ms)
        return round(nbytes / (best * 1e-3) / 1e9, 1)

    copy_gbs = rate(lambda: y.copy_(x))
    scale_gbs = rate(lambda: y.mul_(-1.0))
    return {"copy_gbs": copy_gbs, "scale_in_place_gbs": scale_gbs, "bytes": nbytes,
            "kernels": "torch Tensor.copy_ and Tensor.mul_ (in place) over the 1 GiB sweep buffers, best of 3x"
                       f"{reps} launches, outside the timed region"}


def kernel_label(k: dict) -> str:
    """Name of one plan's kernel in the launch-timing log, as the profile
    summaries name it: precision, kind, length, E, width (C sub-signals of a
    tile or W waves of a single pass), ABFT mode."""
    w = "W" if k["kind"] in ("single", "ragged") else "C"
    return f"{k['precision']} {k['kind']} Ns={k['Ns']} E={k['E']} {w}={k['width']} ft={k['ft']}"


def kernel_fingerprint() -> str:
    """Hash of the kernel sources and the tuning table (which sets the bytes
    per launch), to match stored counter readings to the library being timed."""
    import hashlib
    m = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2412_05824_amd")
    for f in ("csrc/tfft_device.hpp", "csrc/tfft_kernels.hpp", "csrc/inst_fp32_single.hip",
              "csrc/inst_fp32_single_e8.hip",
              "csrc/inst_fp32_single_stream.hip", "csrc/inst_fp32_single_16k.hip",
              "csrc/inst_fp32_tiles.hip", "csrc/inst_fp32_tiles_narrow.hip",
              "csrc/inst_fp32_tiles_e8.hip", "csrc/inst_fp32_tiles_wide.hip", "csrc/inst_fp32_three.hip",
              "tuning/mi355x.json"):
        path = os.path.join(pkg, f)
        if os.path.exists(path):
            with open(path, "rb") as fh:
                m.update(fh.read())
    return m.hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--sizes", type=str, default="", help="comma list of log2 N (default 6..22)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extra", action="store_true", help="skip the off/injection sweep")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-ragged", action="store_true", help="skip the ragged-batch comparison")
    p.add_argument("--no-fp64", action="store_true", help="skip the fp64 forward+inverse sweep")
    p.add_argument("--no-autograd", action="store_true", help="skip the autograd step")
    p.add_argument("--no-three", action="store_true", help="skip the three-pass sweep (N = 2^23..2^29)")
    p.add_argument("--ragged-only", action="store_true",
                   help="only run the ragged-batch comparison (for profiling its kernels)")
    p.add_argument("--ragged-signals", type=int, default=10000)
    p.add_argument("--no-ragged-small", action="store_true",
                   help="skip the small-signal ragged batch (profiles of the 10,000-signal workload alone)")
    p.add_argument("--copy-ref", action="store_true",
                   help="only run a plain 1 GiB device copy (reference for counter scaling)")
    p.add_argument("--study", choices=("roc", "ablation", "offline", "stepwise"), default=None,
                   help="only run a study and print its JSON line: roc (detection vs false alarm over "
                        "the threshold), ablation (ABFT granularity x transactions per group), offline "
                        "(fused vs unfused ABFT), stepwise (the plain transform from per-stage radix-2 "
                        "launches to the tuned plans)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        # signals are independent: several GPUs would each run this
        # benchmark on their share of the batch, with no exchange
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1 "
                                   "(signals shard across GPUs with no communication)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2412_05824_amd as tf
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    if args.ragged_only:
        print(json.dumps({"ragged": ragged_compare(tf, synth, np, torch, dev, args)}), flush=True)
        return
    if args.study:
        fn = {"roc": lambda: roc_study(tf, torch, np, dev),
              "ablation": lambda: ablation_study(tf, torch, dev),
              "offline": lambda: offline_study(tf, torch, dev),
              "stepwise": lambda: stepwise_study(tf, torch, dev)}[args.study]
        print(json.dumps({"study": args.study, **fn()}), flush=True)
        return
    if args.copy_ref:
        src = torch.zeros(TOTAL_ELEMS, dtype=torch.complex64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_per_launch": 2 * TOTAL_ELEMS * 8}), flush=True)
        return
    logs = [int(s) for s in args.sizes.split(",") if s] if args.sizes else list(range(6, 23))
    sizes = [1 << k for k in logs if tf.supported(1 << k, torch.complex64)]
    skipped = [1 << k for k in logs if (1 << k) not in sizes]

    # one seeded 1 GiB input, viewed as [2^27 / N, N] for every N
    t0 = time.time()
    x_host = synth.signals(1, TOTAL_ELEMS, seed=2000, dtype=np.complex64).reshape(-1)
    x = torch.from_numpy(x_host).to(dev)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    print(f"# input ready in {time.time() - t0:.1f}s; sizes {sizes}", file=sys.stderr, flush=True)

    def launch(N, ft):
        xv = x.view(-1, N)
        yv = y.view(-1, N)
        tf.fft_c2c(xv, dir=tf.FORWARD, ft_mode=ft, out=yv, counts=counts)

    for N in sizes:
        tf.prepare(N, torch.complex64, tf.FT_CORRECT)
        tf.prepare(N, torch.complex64, tf.FT_OFF)

    def time_sweep(ft, steps, warmup, per_kernel=None):
        for _ in range(warmup):
            for N in sizes:
                launch(N, ft)
        torch.cuda.synchronize()
        ev = {N: [] for N in sizes}
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(steps):
            for N in sizes:
                if per_kernel is not None:
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    launch(N, ft)
                    b.record(stream)
                    ev[N].append((a, b))
                else:
                    launch(N, ft)
        end.record(stream)
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(end)
        if per_kernel is not None:
            for N in sizes:
                per_kernel[N] = sum(a.elapsed_time(b) for a, b in ev[N]) / len(ev[N])
        return total_ms

    # ---- timed region: K steps of the ABFT sweep ----
    from paper_2412_05824_amd import _lib
    lib = _lib.load()
    torch.cuda.synchronize()
    per_kernel_ms = {}
    # Warmup steps with HIP events around every kernel launch: the per-kernel
    # table and the choice of the kernel that takes most of the step.  In the
    # timed steps only that kernel's launches are bracketed (events cost the
    # stream a few microseconds each: on every launch, 4 % of the step).
    lib.tfft_profile_only(-1, -1, -1, -1, -1)
    lib.tfft_profile(1)
    _lib.profile_read()
    for _ in range(args.warmup):
        for N in sizes:
            launch(N, tf.FT_CORRECT)
    torch.cuda.synchronize()
    kernels = [k for k in _lib.profile_read() if k["ft"] >= 2]
    if kernels:
        k0 = max(kernels, key=lambda k: k["total_ms"])
        _lib.check(lib.tfft_profile_only(0 if k0["precision"] == "fp32" else 1,
                                         ("single", "colpass", "rowpass", "ragged", "colpass3", "rowpass3").index(k0["kind"]),
                                         k0["Ns"], k0["ft"], k0["variant"]), "tfft_profile_only")
    total_ms = time_sweep(tf.FT_CORRECT, args.steps, 0, per_kernel=per_kernel_ms)
    timed = [k for k in _lib.profile_read() if k["ft"] >= 2]
    lib.tfft_profile(0)
    lib.tfft_profile_only(-1, -1, -1, -1, -1)
    kernels_from = "warmup steps (every launch timed)"
    if not kernels:   # no warmup: every launch was timed in the timed steps
        kernels, kernels_from = timed, "timed steps"
    ms_per_step = total_ms / args.steps
    bytes_per_step = sum(2 * TOTAL_ELEMS * 8 for _ in sizes)
    value = bytes_per_step / (ms_per_step * 1e-3) / 1e9
    c_clean = tf.counts_dict(counts)

    sweep = {}
    for N in sizes:
        sweep[N] = {"ft_ms": per_kernel_ms[N],
                    "ft_gbs": 2 * TOTAL_ELEMS * 8 / (per_kernel_ms[N] * 1e-3) / 1e9}

    # ---- context (outside the timed region): ABFT off, and under injection ----
    if not args.no_extra:
        off_ms = {}
        time_sweep(tf.FT_OFF, max(3, args.steps // 2), 1, per_kernel=off_ms)
        rng = np.random.default_rng(2024)
        for N in sizes:
            ab_ft, ab_off = ab_overhead(tf, torch, stream, launch, N)
            sweep[N].update({
                "off_ms": off_ms[N],
                "off_gbs": 2 * TOTAL_ELEMS * 8 / (off_ms[N] * 1e-3) / 1e9,
                "ft_overhead_pct": 100.0 * (ab_ft / ab_off - 1.0),
                "ab_ft_ms": ab_ft, "ab_off_ms": ab_off,
                "sweep_overhead_pct": 100.0 * (per_kernel_ms[N] / off_ms[N] - 1.0),
                **injection_run(tf, torch, np, stream, counts, launch, y, N, TOTAL_ELEMS // N,
                                per_kernel_ms[N], rng, torch.complex64),
            })

    # ---- what plain streaming kernels reach on this GPU (context) ----
    stream_ref = None if args.no_extra else streaming_reference(torch, stream, x, y)

    # ---- ragged batch: one persistent launch vs one launch per length ----
    ragged = None
    if not args.no_ragged:
        ragged = ragged_compare(tf, synth, np, torch, dev, args)

    three = None if args.no_three else three_pass_sweep(tf, torch, np, dev, args, x)
    fp64 = None if args.no_fp64 else fp64_sweep(tf, torch, dev, args)
    grad = None if args.no_autograd else autograd_step(tf, torch, dev, args)

    # ---- roofline of the kernel that takes most of the step (timed steps) ----
    dom = max(timed, key=lambda k: k["total_ms"])
    dom_name = kernel_label(dom)
    dom_avg_ms = dom["total_ms"] / dom["launches"]
    dom_bytes = dom["bytes"] / dom["launches"]
    achieved = dom_bytes / (dom_avg_ms * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        # counters taken on other kernel sources do not describe this library
        tj = json.load(open(tpath))
        if tj.get("kernel_source_sha256_16") == kernel_fingerprint():
            rec = tj.get("kernels", {}).get(dom_name)
            traffic = rec["traffic_bytes"] if rec else None

    # ---- CPU oracle baseline on a bounded sample (rank 0, N=1) ----
    cpu = None
    if not args.no_cpu:
        import oracle
        # the host cores this process may run on, at most the 16-core share a
        # one-GPU job has on the benchmark hosts
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = max(1, min(16, avail))
        per_n_elems = 1 << 26
        t_total = 0.0
        bytes_total = 0
        done = []
        budget = args.cpu_seconds
        for N in sizes:
            nsig = max(1, per_n_elems // N)
            xs = x_host[: nsig * N].reshape(nsig, N)
            t1 = time.perf_counter()
            oracle.fft(xs, threads=threads)
            dt = time.perf_counter() - t1
            t_total += dt
            bytes_total += 2 * nsig * N * 8
            done.append(N)
            if t_total > budget:
                break
        cpu = {"value": bytes_total / t_total / 1e9, "unit": "GB/s", "cores": threads,
               "kind": "oracle", "nproc": os.cpu_count(), "affinity": avail, "cpu_model": cpu_model(),
               "sample": f"{per_n_elems} elements per N for N in {done[0]}..{done[-1]} "
                         f"({len(done)} sizes, {t_total:.1f}s, fp64 recursive radix-2 FFT)"}

    out = {
        "metric": "batched C2C FFT GB/s & % HBM peak (FP32/FP64); ABFT overhead %; ragged vs per-size",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fp32 complex64 forward C2C FFT sweep N=2^6..2^22, "
                               "batch=2^27/N (1 GiB/buffer), two-side ABFT on",
                   "sizes": sizes, "sizes_missing": skipped, "ft_mode": "correct",
                   "overhead": "sweep[N].ft_overhead_pct: ABFT correct vs off on the length's own tuned "
                               "routes, alternating rounds of 10 launches, best round of each "
                               "(ab_ft_ms, ab_off_ms); sweep_overhead_pct: the timed ABFT sweep's "
                               "launch time over the later plain sweep's",
                   "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": f"k_fft {dom_name}",
                     "avg_launch_us": round(dom_avg_ms * 1e3, 2),
                     "bytes_per_launch": dom_bytes,
                     "share_of_step": round(dom["total_ms"] / total_ms, 3)},
        "kernels": [{"label": kernel_label(k), **k, "avg_us": round(1e3 * k["total_ms"] / k["launches"], 2),
                     "gbs": round(k["bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1)} for k in
                    sorted(kernels, key=lambda k: -k["total_ms"])],
        "kernels_from": kernels_from,
        "cpu_baseline": cpu,
        "streaming_reference": stream_ref,
        "clean_counts": c_clean,
        "sweep": {str(k): v for k, v in sweep.items()},
        "ragged": ragged,
        "fp64_sweep": fp64,
        "three_pass": three,
        "autograd": grad,
    }
    print(json.dumps(out), flush=True)


def flip_value(v: complex, part: int, bit: int, real_dtype) -> complex:
    """v with one bit of its real (part 0) or imaginary part flipped, as
    stored in binary32 / binary64 (the injected fault, seen from the host)."""
    import numpy as np
    a = np.array([v.real, v.imag], dtype=real_dtype)
    u = a.view(np.uint32 if real_dtype == np.float32 else np.uint64)
    u[part] ^= (1 << bit)
    return complex(float(a[0]), float(a[1]))


def ab_overhead(tf, torch, stream, launch, N, rounds=3, reps=10):
    """ABFT correct against ABFT off on one length under the same conditions:
    rounds of `reps` back-to-back launches of each mode, alternating (HIP
    events around each round), best round of each mode; ms per launch."""
    best = {}
    for ft in (tf.FT_OFF, tf.FT_CORRECT):
        launch(N, ft)
    torch.cuda.synchronize()
    for _ in range(rounds):
        for ft in (tf.FT_OFF, tf.FT_CORRECT):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                launch(N, ft)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            best[ft] = min(best.get(ft, ms), ms)
    return best[tf.FT_CORRECT], best[tf.FT_OFF]


def injection_run(tf, torch, np, stream, counts, launch, y, N, batch, ft_ms, rng, dtype,
                  n_launch=100, direction=None):
    """Two windows of n_launch ABFT launches back to back (HIP events around
    each launch): fault-free, then with one (seeded) launch carrying a
    single-bit flip in a random output element.  Reports the mean launch
    time of both, the injection overhead (one window over the other), the
    extra time of the launch that carried the flip over the window's median,
    the counts, and the flip: its size relative to the hit signal's norm,
    whether it is significant (an uncorrected flip of that size would take
    the signal past the acceptance tolerance) and the hit signal's relative
    distance, after correction, to its fault-free output."""
    fp32 = dtype == torch.complex64
    tol = 2e-6 if fp32 else 1e-13
    nbits = 31 if fp32 else 63
    counts.zero_()
    hit = int(rng.integers(0, n_launch))
    sig, elem = int(rng.integers(0, batch)), int(rng.integers(0, N))
    part, bit = int(rng.integers(0, 2)), int(rng.integers(0, nbits))
    yv = y.view(-1, N)
    kept = torch.empty(N, dtype=dtype, device=y.device)

    def window(inject):
        # n_launch ABFT launches back to back, each bracketed by events; with
        # inject, launch `hit` carries the flip
        evs = []
        for i in range(n_launch):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            if inject and i == hit:
                tf.inject_arm(sig, elem, part, bit, dtype=dtype)
            a.record(stream)
            launch(N, tf.FT_CORRECT)
            b.record(stream)
            evs.append((a, b))
            if inject and i == hit:
                kept.copy_(yv[sig])   # the corrected signal, before later launches overwrite it
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    # the fault-free window is the baseline, timed the same way in the same
    # context (back-to-back launches of one length)
    base = window(False)
    counts.zero_()
    times = window(True)
    base_ms = sum(base) / n_launch
    inj_ms = sum(times) / n_launch
    others = sorted(t for i, t in enumerate(times) if i != hit)
    hit_extra_us = 1e3 * (times[hit] - others[len(others) // 2])
    cd = tf.counts_dict(counts)
    launch(N, tf.FT_OFF)                      # fault-free output of the same input
    torch.cuda.synchronize()
    clean = yv[sig].to(torch.complex128)
    norm = torch.linalg.vector_norm(clean).item()
    yc = complex(clean[elem].item())
    delta = abs(flip_value(yc, part, bit, np.float32 if fp32 else np.float64) - yc)
    delta_rel = delta / norm if norm > 0 else float("inf")
    after = torch.linalg.vector_norm(kept.to(torch.complex128) - clean).item() / norm
    return {
        "inj_ms": inj_ms,
        "inj_base_ms": base_ms,
        "inj_overhead_pct": 100.0 * (inj_ms / base_ms - 1.0),
        "inj_hit_launch_extra_us": round(hit_extra_us, 2),
        "inj_flip": {"launch": hit, "signal": sig, "element": elem, "part": part, "bit": bit,
                     "delta_rel": delta_rel if math.isfinite(delta_rel) else "inf",
                     "significant": not (delta_rel <= tol),
                     "hit_signal_rel_after": after,
                     "hit_signal_within_tol": after <= tol},
        "inj_counts": {k: cd[k] for k in ("detected", "corrected", "rebuilt", "uncorrectable")},
    }


def three_pass_sweep(tf, torch, np, dev, args, x1g):
    """complex64 forward transforms of N = 2^23..2^29 on the three-pass
    route (three launches per chunk of signals), batch 2^27 / N (at least
    one signal; the headline input for N <= 2^27, a seeded device input
    beyond), ABFT off and correct, with the per-pass kernel times from the
    launch-timing log and one seeded single-bit flip in each pass checked
    against the fault-free output.  GB/s counts the transform's input and
    output once (2 N batch 8 bytes); each pass moves that much again."""
    from paper_2412_05824_amd import _lib
    lib = _lib.load()
    dt = torch.complex64
    counts = tf.new_counts(dev)
    rng = np.random.default_rng(2300)
    reps = max(3, args.steps // 2)
    out = {}
    for lg in range(23, 30):
        N = 1 << lg
        if not tf.supported(N, dt):
            continue
        info = tf.route_info(N, dt)
        if N <= TOTAL_ELEMS:
            x = x1g.view(-1, N)
        else:
            g = torch.Generator(device=dev)
            g.manual_seed(2300 + lg)
            x = (torch.rand(N, 2, dtype=torch.float32, device=dev, generator=g) * 2 - 1).view(dt).view(1, N)
        y = torch.empty_like(x)
        batch = x.shape[0]
        tf.prepare(N, dt, tf.FT_CORRECT, batch=batch, device=dev)
        tf.prepare(N, dt, tf.FT_OFF, batch=batch, device=dev)
        ms = {}
        counts.zero_()
        for ft in (tf.FT_OFF, tf.FT_CORRECT):
            for _ in range(max(1, args.warmup)):
                tf.fft_c2c(x, ft_mode=ft, out=y, counts=counts)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                tf.fft_c2c(x, ft_mode=ft, out=y, counts=counts)
            b.record()
            torch.cuda.synchronize()
            ms[ft] = a.elapsed_time(b) / reps
        clean = tf.counts_dict(counts)["detected"]
        # per-pass kernel times (every launch bracketed by events)
        lib.tfft_profile_only(-1, -1, -1, -1, -1)
        lib.tfft_profile(1)
        _lib.profile_read()
        for _ in range(reps):
            tf.fft_c2c(x, ft_mode=tf.FT_CORRECT, out=y, counts=counts)
        torch.cuda.synchronize()
        passes = [{"kind": k["kind"], "Ns": k["Ns"], "E": k["E"], "width": k["width"], "launches": k["launches"],
                   "avg_us": round(1e3 * k["total_ms"] / k["launches"], 2),
                   "gbs": round(k["bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1)}
                  for k in _lib.profile_read()]
        lib.tfft_profile(0)
        # one flip per pass, the hit signal against its fault-free output
        tf.fft_c2c(x, ft_mode=tf.FT_OFF, out=y)
        flips = []
        for pass_ in (0, 1, 2):
            sig, elem = int(rng.integers(0, batch)), int(rng.integers(0, N))
            part, bit = int(rng.integers(0, 2)), int(rng.integers(20, 31))
            ref = y[sig].clone()
            counts.zero_()
            tf.inject_arm(sig, elem, part, bit, dtype=dt, pass_=pass_)
            yi = torch.empty_like(y)
            tf.fft_c2c(x, ft_mode=tf.FT_CORRECT, out=yi, counts=counts)
            torch.cuda.synchronize()
            c = tf.counts_dict(counts)
            after = (torch.linalg.vector_norm((yi[sig] - ref).to(torch.complex128)).item() /
                     torch.linalg.vector_norm(ref.to(torch.complex128)).item())
            flips.append({"pass": pass_, "signal": sig, "element": elem, "part": part, "bit": bit,
                          "counts": {k: c[k] for k in ("detected", "corrected", "rebuilt", "uncorrectable")},
                          "hit_signal_rel_after": after, "hit_signal_within_tol": after <= 2e-6,
                          "others_unchanged": bool(torch.equal(torch.cat([yi[:sig], yi[sig + 1:]]),
                                                               torch.cat([y[:sig], y[sig + 1:]])))})
            del yi
        nbytes = 2 * N * batch * 8
        out[str(N)] = {"route": [info["N1"], info["N2"], info["N3"]], "batch": batch,
                       "ft_ms": round(ms[tf.FT_CORRECT], 4), "off_ms": round(ms[tf.FT_OFF], 4),
                       "ft_gbs": round(nbytes / (ms[tf.FT_CORRECT] * 1e-3) / 1e9, 1),
                       "off_gbs": round(nbytes / (ms[tf.FT_OFF] * 1e-3) / 1e9, 1),
                       "ft_overhead_pct": round(100.0 * (ms[tf.FT_CORRECT] / ms[tf.FT_OFF] - 1.0), 1),
                       "clean_detected": clean, "passes": passes, "flips": flips}
        print(f"# three-pass N=2^{lg}: {out[str(N)]['ft_gbs']} GB/s ABFT on, "
              f"{out[str(N)]['off_gbs']} off", file=sys.stderr, flush=True)
        del y
        if N > TOTAL_ELEMS:
            del x
        torch.cuda.empty_cache()
    return {"workload": "complex64 forward C2C, N=2^23..2^29 as three launches (column pass N1, column "
                        "pass N2 with the outer twiddle, row pass N3 with the transposed store), "
                        "batch=max(1, 2^27/N), inputs U[-1,1), ABFT correct vs off, one seeded flip per pass",
            "per_n": out}


def fp64_sweep(tf, torch, dev, args):
    """complex128 forward+inverse sweep with ABFT off / correct and seeded
    flips; inputs standard normal, generated on the device from a seed."""
    import numpy as np
    total = 1 << 26                              # 1 GiB of complex128
    g = torch.Generator(device=dev)
    g.manual_seed(3000)
    x = torch.randn(total, 2, dtype=torch.float64, device=dev, generator=g).view(torch.complex128).view(-1)
    y = torch.empty_like(x)
    counts = tf.new_counts(dev)
    rng = np.random.default_rng(3001)
    reps = max(3, args.steps // 2)
    out = {}
    for lg in range(6, 21):
        N = 1 << lg
        if not tf.supported(N, torch.complex128):
            continue
        xv, yv = x.view(-1, N), y.view(-1, N)
        ms, ms_fwd, ms_inv = {}, {}, {}
        counts.zero_()   # the previous length's injected flips are counted already
        for ft in (tf.FT_OFF, tf.FT_CORRECT):
            # a round trip per step (the in-place inverse brings the forward
            # output back to the input's scale), each launch timed on its own
            def step(ev=None):
                if ev is not None:
                    ev[0].record()
                tf.fft_c2c(xv, dir=tf.FORWARD, ft_mode=ft, out=yv, counts=counts)
                if ev is not None:
                    ev[1].record()
                tf.fft_c2c(yv, dir=tf.INVERSE, ft_mode=ft, out=yv, counts=counts)
                if ev is not None:
                    ev[2].record()
            for _ in range(max(1, args.warmup)):
                step()
            torch.cuda.synchronize()
            evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
            for ev in evs:
                step(ev)
            torch.cuda.synchronize()
            ms_fwd[ft] = sum(ev[0].elapsed_time(ev[1]) for ev in evs) / reps
            ms_inv[ft] = sum(ev[1].elapsed_time(ev[2]) for ev in evs) / reps
            ms[ft] = ms_fwd[ft] + ms_inv[ft]
        # the fault-free runs above must not have counted anything
        clean = tf.counts_dict(counts)
        # seeded flips: one in a forward and one in an inverse launch; the hit
        # signal, after correction, against its fault-free output
        counts.zero_()
        flips = []
        for d in (tf.FORWARD, tf.INVERSE):
            sig, elem = int(rng.integers(0, total // N)), int(rng.integers(0, N))
            part, bit = int(rng.integers(0, 2)), int(rng.integers(0, 63))
            tf.inject_arm(sig, elem, part, bit, dtype=torch.complex128)
            tf.fft_c2c(xv, dir=d, ft_mode=tf.FT_CORRECT, out=yv, counts=counts)
            kept = yv[sig].clone()
            tf.fft_c2c(xv, dir=d, ft_mode=tf.FT_OFF, out=yv)
            ref = yv[sig]
            norm = torch.linalg.vector_norm(ref).item()
            yc = complex(ref[elem].item())
            delta_rel = abs(flip_value(yc, part, bit, np.float64) - yc) / norm
            after = torch.linalg.vector_norm(kept - ref).item() / norm
            flips.append({"dir": d, "signal": sig, "element": elem, "part": part, "bit": bit,
                          "delta_rel": delta_rel if math.isfinite(delta_rel) else "inf",
                          "significant": not (delta_rel <= 1e-13),
                          "hit_signal_rel_after": after, "hit_signal_within_tol": after <= 1e-13})
        torch.cuda.synchronize()
        c = tf.counts_dict(counts)
        bytes_one = 2 * total * 16                   # one transform: read + write
        gbs = lambda t: round(bytes_one / (t * 1e-3) / 1e9, 1)
        out[str(N)] = {"ft_gbs": gbs(ms_fwd[2]),
                       "off_gbs": gbs(ms_fwd[0]),
                       "ft_overhead_pct": round(100.0 * (ms_fwd[2] / ms_fwd[0] - 1.0), 1),
                       "inverse_in_place": {"ft_gbs": gbs(ms_inv[2]), "off_gbs": gbs(ms_inv[0]),
                                            "ft_overhead_pct": round(100.0 * (ms_inv[2] / ms_inv[0] - 1.0), 1)},
                       "round_trip_ft_overhead_pct": round(100.0 * (ms[2] / ms[0] - 1.0), 1),
                       "clean_detected": clean["detected"],
                       "flips": flips,
                       "counts": {k: c[k] for k in ("detected", "corrected", "rebuilt", "uncorrectable")}}
    del x, y
    torch.cuda.empty_cache()
    return {"workload": "complex128 forward (out of place; ft_gbs, off_gbs, ft_overhead_pct) then inverse "
                        "(in place, the in-place correcting kernels; inverse_in_place), N=2^6..2^20, batch=2^26/N "
                        "(1 GiB), inputs N(0,1) from a device generator (seed 3000), ABFT correct vs off, "
                        "each launch timed with HIP events, 2 seeded flips per N",
            "per_n": out}


def autograd_step(tf, torch, dev, args):
    """loss = sum(w * |FFT(x)|^2), x complex64 [16384, 4096]: forward and the
    ABFT-protected adjoint; ms per step and algorithmic GB/s of the two FFTs."""
    B, N = 16384, 4096
    g = torch.Generator(device=dev)
    g.manual_seed(4000)
    x = (torch.rand(B, N, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(B, N)
    x.requires_grad_(True)
    w = torch.rand(B, N, device=dev, generator=g)
    reps = max(3, args.steps // 2)

    def step():
        x.grad = None
        y = tf.fft(x, ft_mode=tf.FT_CORRECT)
        loss = (w * (y.real * y.real + y.imag * y.imag)).sum()
        loss.backward()
        return loss

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    fft_bytes = 2 * 2 * B * N * 8                  # forward + adjoint, read + write
    out = {"workload": "loss = sum(w*|FFT(x)|^2), x complex64 [16384, 4096], w U[0,1), ABFT correct",
           "ms_per_step": round(ms, 4),
           "fft_gbs_in_step": round(fft_bytes / (ms * 1e-3) / 1e9, 1)}
    del x, w
    torch.cuda.empty_cache()
    return out


def ragged_compare(tf, synth, np, torch, dev, args):
    """Time the ragged workload in its three forms; returns a dict for the JSON
    line, with a second, small-signal batch (lengths 64..3072) as context."""
    out = ragged_one(tf, synth, np, torch, dev, args,
                     [int(n) for n in synth.ragged_sizes(args.ragged_signals, seed=5)],
                     f"{args.ragged_signals} fp32 signals, lengths uniform over 2^k and 3*2^k, "
                     f"6<=k<=16 (seed 5)")
    if args.no_ragged_small:
        return out
    small_menu = [n for n in synth.RAGGED_SIZES if n <= 3072]
    out["small_signals"] = ragged_one(
        tf, synth, np, torch, dev, args,
        [int(n) for n in synth.ragged_sizes(2000, seed=6, menu=small_menu)],
        "2000 fp32 signals, lengths uniform over 2^k and 3*2^k, 6<=k<=10 (seed 6)")
    return out


def ragged_one(tf, synth, np, torch, dev, args, sizes, desc):
    """One ragged batch in its three forms."""
    total = int(sum(sizes))
    x = torch.from_numpy(synth.signals(1, total, seed=2005).reshape(-1)).to(dev)
    y = torch.empty_like(x)
    plan = tf.RaggedPlan(sizes, device=dev)
    counts = tf.new_counts(dev)
    reps = max(3, args.steps)

    def timed(fn):
        for _ in range(max(1, args.warmup)):
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

    def captured(mode):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan(x, out=y, ft_mode=tf.FT_CORRECT, counts=counts, mode=mode)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan(x, out=y, ft_mode=tf.FT_CORRECT, counts=counts, mode=mode)
        return g

    res = {}
    for mode in ("persistent", "per_size"):
        res[f"{mode}_eager_ms"] = timed(lambda: plan(x, out=y, ft_mode=tf.FT_CORRECT, counts=counts,
                                                     mode=mode))
        g = captured(mode)
        res[f"{mode}_graph_ms"] = timed(g.replay)
        del g
    off_ms = timed(lambda: plan(x, out=y, ft_mode=tf.FT_OFF, mode="persistent"))
    info = plan.info(device_state=True)
    c = tf.counts_dict(counts)
    bytes_alg = 2.0 * total * 8
    best_per_size = min(res["per_size_eager_ms"], res["per_size_graph_ms"])
    out = {
        "workload": f"{desc}, {total} elements, forward, ABFT correct",
        "elements": total,
        "work_items": info["items"],
        "persistent_grid": info["grid"],
        **{k: round(v, 4) for k, v in res.items()},
        "persistent_ft_off_ms": round(off_ms, 4),
        "gbs_persistent_graph": round(bytes_alg / (res["persistent_graph_ms"] * 1e-3) / 1e9, 1),
        "gbs_per_size_eager": round(bytes_alg / (res["per_size_eager_ms"] * 1e-3) / 1e9, 1),
        "speedup_vs_per_size_eager": round(res["per_size_eager_ms"] / res["persistent_graph_ms"], 3),
        "speedup_vs_best_per_size": round(best_per_size / res["persistent_graph_ms"], 3),
        "detected": c["detected"],
        "err_launches": info["err_launches"],
    }
    plan.close()
    del x, y
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Studies (outside the headline step): ROC of the detection threshold and the
# ABFT granularity ablation.
# ---------------------------------------------------------------------------

ROC_KAPPAS = (0.125, 0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 32.0, 64.0, 256.0)


def roc_study(tf, torch, np, dev, N=1024, n_clean=2000, n_inj=1000, kappas=ROC_KAPPAS):
    """Detection vs false alarm over the threshold factor kappa (Sec. 5.3
    "Error Injection Analysis": 2000 normally distributed signals, 1000 of
    them with one flipped bit of one value; the paper sweeps its threshold
    delta, here tau = kappa u sqrt(N log2 N) sqrt(nu)).  Each signal is
    checked on its own (per-transaction granularity, one transaction per
    group).  Flips are drawn once (signal, element, real/imag, any bit of
    the binary32/binary64 value) and replayed for every kappa; a flip is
    significant when it moves its signal by more than the acceptance
    tolerance (relative L2), the ones the check must not miss."""
    out = {}
    for dtype, prec, nbits, tol in ((torch.complex64, "fp32", 32, 2e-6), (torch.complex128, "fp64", 64, 1e-13)):
        rdt = torch.float32 if prec == "fp32" else torch.float64
        g = torch.Generator(device=dev)
        g.manual_seed(6000)
        x = torch.randn(n_clean, N, 2, dtype=rdt, device=dev, generator=g).view(dtype).view(n_clean, N)
        y = torch.empty_like(x)
        tf.fft_c2c(x, ft_mode=tf.FT_OFF, out=y)
        yc = y.to(torch.complex128).cpu().numpy()
        rng = np.random.default_rng(6001)
        flips = []
        for _ in range(n_inj):
            s, e, part, bit = (int(rng.integers(0, n_clean)), int(rng.integers(0, N)),
                               int(rng.integers(0, 2)), int(rng.integers(0, nbits)))
            v = complex(yc[s, e])
            delta = abs(flip_value(v, part, bit, np.float32 if prec == "fp32" else np.float64) - v)
            rel = delta / float(np.linalg.norm(yc[s]))
            flips.append((s, e, part, bit, not (rel <= tol)))
        n_sig = sum(1 for f in flips if f[4])
        T0, k0 = tf.get_tuning(N, dtype)
        gran0 = tf.route_info(N, dtype)["gran"]
        counts = tf.new_counts(dev)
        pts = []
        try:
            tf.set_granularity(N, dtype, 1)
            for kappa in kappas:
                tf.set_tuning(N, dtype, 1, kappa)
                counts.zero_()
                tf.fft_c2c(x, ft_mode=tf.FT_DETECT, out=y, counts=counts)
                fa = tf.counts_dict(counts)["detected"]
                det = det_sig = 0
                for s, e, part, bit, sig in flips:
                    counts.zero_()
                    tf.inject_arm(0, e, part, bit, dtype=dtype)
                    tf.fft_c2c(x[s:s + 1], ft_mode=tf.FT_DETECT, out=y[:1], counts=counts)
                    hit = tf.counts_dict(counts)["detected"] > 0
                    det += hit
                    det_sig += hit and sig
                pts.append({"kappa": kappa, "false_alarm_rate": fa / n_clean, "detection_rate": det / n_inj,
                            "detection_rate_significant": det_sig / max(1, n_sig)})
        finally:
            tf.set_tuning(N, dtype, T0, k0)
            tf.set_granularity(N, dtype, gran0)
        out[prec] = {"N": N, "clean_signals": n_clean, "injected": n_inj, "significant": n_sig,
                     "default_kappa": k0, "points": pts}
        del x, y
    torch.cuda.empty_cache()
    return {"workload": f"{n_clean} N(0,1) signals of {N} points per precision (seed 6000), "
                        f"{n_inj} single-bit flips (seed 6001), FT_DETECT per transaction, T = 1",
            **out}


def ablation_study(tf, torch, dev, reps=5):
    """ABFT granularity x transactions per group (Sec. 4.2-4.3; Table 2's
    stepwise comparison): overhead of the correcting kernels over the plain
    ones on a 1 GiB batch, per length, for the thread level (every radix-R
    DFT checked in registers; single-pass lengths), the check once per group
    (location code) at T = 1..32 and per transaction at T = 1..16.  The route of each length stays the tuned one;
    rows whose group size breaks the accuracy bound are marked (those
    settings are never chosen by the autotuner)."""
    from paper_2412_05824_amd import autotune
    rows = []
    for dtype, prec, lens in ((torch.complex64, "fp32", (1024, 4096, 1 << 16, 1 << 20)),
                              (torch.complex128, "fp64", (1024, 4096, 1 << 16))):
        esize = 8 if prec == "fp32" else 16
        total = (1 << 30) // esize
        rdt = torch.float32 if prec == "fp32" else torch.float64
        g = torch.Generator(device=dev)
        g.manual_seed(6100)
        x = (torch.rand(total, 2, dtype=rdt, device=dev, generator=g) * 2 - 1).view(dtype).view(-1)
        y = torch.empty_like(x)
        counts = tf.new_counts(dev)
        for N in lens:
            xv, yv = x.view(-1, N), y.view(-1, N)
            T0, k0 = tf.get_tuning(N, dtype)
            info0 = tf.route_info(N, dtype)
            gran0 = info0["gran"]

            def tm(ft):
                run = lambda: tf.fft_c2c(xv, ft_mode=ft, out=yv, counts=counts)
                for _ in range(2):
                    run()
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                best = 1e30
                for _ in range(3):
                    a.record()
                    for _ in range(reps):
                        run()
                    b.record()
                    torch.cuda.synchronize()
                    best = min(best, a.elapsed_time(b) / reps)
                return best
            try:
                offs = []
                for T in (1, 2):
                    tf.set_tuning(N, dtype, T, 0)
                    offs.append(tm(tf.FT_OFF))
                off = min(offs)
                s_route = autotune.steps(N, 1 if info0["passes"] == 1 else info0["N1"])
                if info0["passes"] == 1:
                    # thread level: every radix-R DFT checked in registers
                    counts.zero_()
                    ms = tm(tf.FT_THREAD)
                    rows.append({"precision": prec, "N": N, "granularity": "thread", "T": 1,
                                 "ft_ms": round(ms, 4), "off_ms": round(off, 4),
                                 "overhead_pct": round(100 * (ms / off - 1), 1),
                                 "within_accuracy_bound": True,
                                 "detected": tf.counts_dict(counts)["detected"]})
                for gran, Ts in ((0, (1, 2, 4, 8, 16, 32)), (1, (1, 2, 4, 8, 16))):
                    tf.set_granularity(N, dtype, gran)
                    seen = set()
                    for T in Ts:
                        tf.set_tuning(N, dtype, T, 0)
                        teff = tf.route_info(N, dtype)["T"]
                        if teff in seen:
                            continue
                        seen.add(teff)
                        counts.zero_()
                        ms = tm(tf.FT_CORRECT)
                        within = gran == 1 or teff <= autotune.max_T(prec, s_route, k0)
                        rows.append({"precision": prec, "N": N, "granularity": "transaction" if gran else "group",
                                     "T": teff, "ft_ms": round(ms, 4), "off_ms": round(off, 4),
                                     "overhead_pct": round(100 * (ms / off - 1), 1),
                                     "within_accuracy_bound": within,
                                     "detected": tf.counts_dict(counts)["detected"]})
            finally:
                tf.set_tuning(N, dtype, T0, k0)
                tf.set_granularity(N, dtype, gran0)
        del x, y
        torch.cuda.empty_cache()
    return {"workload": "1 GiB uniform batch per length, forward, tuned route; plain kernel at its best of T = 1, 2",
            "rows": rows}


def stepwise_study(tf, torch, dev, reps=3):
    """The plain transform (no ABFT) at the four levels of tfft_c2c_stepwise
    (Sec. 5.1's v0 -> v3 chain): 0 one launch per radix-2 stage through
    global memory, 1 all radix-2 stages in one launch through LDS (N <= 8192),
    2 the default plans (radix-16 stages, untuned), 3 the tuned routes.
    complex64 forward, batch 2^27 / N (1 GiB), N = 2^6..2^22; GB/s counts the
    transform's input and output once, GFLOPS 5 N log2 N per signal."""
    total = TOTAL_ELEMS
    g = torch.Generator(device=dev)
    g.manual_seed(2600)
    x = (torch.rand(total, 2, device=dev, generator=g) * 2 - 1).view(torch.complex64).view(-1)
    y = torch.empty_like(x)
    out = {}
    for lg in range(6, 23):
        N = 1 << lg
        xv, yv = x.view(-1, N), y.view(-1, N)
        row = {}
        for level in (0, 1, 2, 3):
            if level == 1 and N > 8192:
                continue
            fn = lambda: tf.fft_c2c_stepwise(xv, level, out=yv)
            fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            row[f"v{level}"] = {"ms": round(ms, 4), "gbs": round(2 * total * 8 / (ms * 1e-3) / 1e9, 1),
                                "gflops": round(5.0 * total * lg / (ms * 1e-3) / 1e9, 1)}
        out[str(N)] = row
        print(f"# stepwise N=2^{lg}: " + ", ".join(f"{k} {v['gbs']} GB/s" for k, v in row.items()),
              file=sys.stderr, flush=True)
    del x, y
    torch.cuda.empty_cache()
    return {"workload": "complex64 forward, batch 2^27/N (1 GiB), inputs U[-1,1), no ABFT; v0 per-stage "
                        "radix-2 launches, v1 radix-2 stages in one launch, v2 default plans, v3 tuned",
            "per_n": out}


def offline_study(tf, torch, dev, reps=5):
    """Fused vs offline two-side ABFT (Sec. 5.2 and Fig. 20's comparison,
    with this library's own plain transform as the base): per length, on a
    1 GiB batch, the plain transform, the fused correcting kernels and the
    offline scheme (tfft_c2c_offline: separate checksum passes, transform of
    the right-side sums, check and fix), without and with one seeded flip in
    a window of 20 launches."""
    rows = []
    for dtype, prec, lens in ((torch.complex64, "fp32", (256, 4096, 1 << 16, 1 << 20, 1 << 22)),
                              (torch.complex128, "fp64", (1024, 1 << 16))):
        esize = 8 if prec == "fp32" else 16
        total = (1 << 30) // esize
        rdt = torch.float32 if prec == "fp32" else torch.float64
        g = torch.Generator(device=dev)
        g.manual_seed(6200)
        x = (torch.rand(total, 2, dtype=rdt, device=dev, generator=g) * 2 - 1).view(dtype).view(-1)
        y = torch.empty_like(x)
        counts = tf.new_counts(dev)
        for N in lens:
            xv, yv = x.view(-1, N), y.view(-1, N)
            batch = xv.shape[0]
            runs = {
                "plain": lambda: tf.fft_c2c(xv, ft_mode=tf.FT_OFF, out=yv),
                "fused": lambda: tf.fft_c2c(xv, ft_mode=tf.FT_CORRECT, out=yv, counts=counts),
                "offline": lambda: tf.fft_c2c_offline(xv, out=yv, counts=counts),
            }
            ms = {}
            for k, fn in runs.items():
                for _ in range(2):
                    fn()
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                best = 1e30
                for _ in range(3):
                    a.record()
                    for _ in range(reps):
                        fn()
                    b.record()
                    torch.cuda.synchronize()
                    best = min(best, a.elapsed_time(b) / reps)
                ms[k] = best
            # one flip in a window of 20 launches, fused and offline
            inj = {}
            for k in ("fused", "offline"):
                counts.zero_()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                for i in range(20):
                    if i == 7:
                        tf.inject_arm(batch // 2, N // 3, 0, 29 if prec == "fp32" else 61, dtype=dtype)
                    runs[k]()
                b.record()
                torch.cuda.synchronize()
                c = tf.counts_dict(counts)
                inj[k] = {"ms": a.elapsed_time(b) / 20, "detected": c["detected"],
                          "repaired": c["corrected"] + c["rebuilt"]}
            rows.append({"precision": prec, "N": N, "plain_ms": round(ms["plain"], 4),
                         "fused_ms": round(ms["fused"], 4), "offline_ms": round(ms["offline"], 4),
                         "fused_overhead_pct": round(100 * (ms["fused"] / ms["plain"] - 1), 1),
                         "offline_overhead_pct": round(100 * (ms["offline"] / ms["plain"] - 1), 1),
                         "fused_inj_overhead_pct": round(100 * (inj["fused"]["ms"] / ms["plain"] - 1), 1),
                         "offline_inj_overhead_pct": round(100 * (inj["offline"]["ms"] / ms["plain"] - 1), 1),
                         "inj_counts": {k: {kk: v[kk] for kk in ("detected", "repaired")} for k, v in inj.items()}})
        del x, y
        torch.cuda.empty_cache()
    return {"workload": "1 GiB uniform batch per length, forward; with injection: one exponent-bit flip "
                        "in a window of 20 launches", "rows": rows}


if __name__ == "__main__":
    main()
