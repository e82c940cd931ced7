/*
 * tfft.h -- C ABI of the MI355X (gfx950) batched complex-to-complex FFT with
 * fused two-side ABFT (algorithm-based fault tolerance).
 *
 * Method: TurboFFT (Wu et al., PPoPP'25, arXiv:2412.05824).
 *   Transform, Sec. 2.2 "DFT and FFT":
 *     forward  y_k = sum_n x_n exp(-2 pi i k n / N)
 *     inverse  x_k = (1/N) sum_n y_n exp(+2 pi i k n / N)
 *   Fault tolerance, Sec. 4.1-4.3: checksums e^T W x (left side) and W X e
 *   (right side, batch sum), location weights 1, 2, ... per signal, detection
 *   by comparing e^T y with (e^T W) x, correction by adding W(Xe) - Ye to the
 *   located signal after the group of transactions ("delayed batched
 *   correction"), under the single-event-upset assumption (Sec. 2.2 fault
 *   model): at most one faulty signal per group.
 *
 * Conventions for every entry point:
 *   - Complex data are interleaved (re, im), batch-major: signal b occupies
 *     elements [b*N, (b+1)*N).  TFFT_FP32 = complex64 (8 bytes per element),
 *     TFFT_FP64 = complex128 (16 bytes per element).
 *   - Pointers named x, y, counts, offsets, sizes are DEVICE pointers owned by
 *     the caller.  hip_stream is a hipStream_t (NULL = the default stream).
 *   - Calls are asynchronous on hip_stream and never synchronise the device.
 *   - Return value: TFFT_OK or a negative tfft_status.  No exception crosses
 *     the ABI.  Detected and corrected soft errors are data (counters), not
 *     error returns.
 *   - The library owns its twiddle and checksum tables, allocated by
 *     tfft_prepare* (or lazily by the first call outside stream capture) and
 *     freed when the library is unloaded.  A call made while hip_stream is
 *     being captured into a graph never allocates: if its tables are missing
 *     it returns TFFT_ECAPTURE.
 */
#ifndef TFFT_H
#define TFFT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFFT_OK = 0,
    TFFT_EINVAL = -1,       /* null pointer, N < 1, batch < 0, unknown enum value */
    TFFT_EUNSUPPORTED = -2, /* size or mode without a compiled kernel */
    TFFT_EALIGN = -3,       /* x or y not aligned to the element size */
    TFFT_EHIP = -4,         /* HIP runtime error, see tfft_last_hip_error() */
    TFFT_ENOMEM = -5,       /* table allocation failed */
    TFFT_ECAPTURE = -6,     /* would allocate during stream capture */
    TFFT_ENOTPREPARED = -7, /* tfft_c2c_noalloc: tables of the length not built yet */
    TFFT_ESCRATCH = -8      /* tfft_c2c_noalloc: one signal exceeds the scratch buffer */
} tfft_status;

enum { TFFT_FORWARD = -1, TFFT_INVERSE = +1 };       /* sign of the exponent */
enum { TFFT_FP32 = 0, TFFT_FP64 = 1 };
enum { TFFT_FT_OFF = 0, TFFT_FT_DETECT = 1, TFFT_FT_CORRECT = 2, TFFT_FT_THREAD = 3 };

/* Device-resident counters, accumulated by every call that is given them
 * (the caller zeroes them).  detected: faulty signals found (a checksum
 * disagreement, or a non-finite / oversized output); corrected: fixed by
 * adding W(Xe)-Ye; rebuilt: fixed by recomputing the located signal as W(Xe)
 * minus the group's other outputs; uncorrectable: detected but not located or
 * not verified (for example two faults in one group under group-level
 * detection); last_signal: global index of the most recently located signal;
 * calib: see tfft_calibration; sched_errors: persistent ragged launches in
 * which a wait gave up (their outputs are not to be trusted); fallback:
 * detections whose location came from re-encoding every signal of the group
 * because the location code D1/D0 was not an index. */
typedef struct {
    unsigned long long detected, corrected, rebuilt, uncorrectable, last_signal;
    unsigned long long calib, sched_errors, fallback;
} tfft_ft_counts;

/* Batched 1-D C2C transform of `batch` signals of length N.
 *   x, y      device buffers of batch*N elements; x == y (in place) allowed,
 *             partial overlap is not.
 *   dir       TFFT_FORWARD or TFFT_INVERSE.
 *   precision TFFT_FP32 or TFFT_FP64.
 *   ft_mode   TFFT_FT_OFF, TFFT_FT_DETECT (one-side check with location) or
 *             TFFT_FT_CORRECT (two-side check, location and correction), or
 *             TFFT_FT_THREAD: thread-level two-side ABFT (Sec. 4.2), the
 *             granularity study's finest form: every radix-R DFT a lane
 *             computes in registers is checked, located and corrected on
 *             its own (threshold kappa u sqrt(R (log2 R + 3)) |v|, kappa of the
 *             length's tuning); the LDS exchanges and twiddle products
 *             between them are not covered.  Single-pass lengths only (the
 *             correcting mode's route; TFFT_EUNSUPPORTED otherwise).  An
 *             armed injection (pass 0) flips output (element / P) mod R of
 *             the first DFT of lane t = element mod P (P lanes per signal)
 *             at stage `stage`, between the DFT and its check.
 *   scale     multiplies every output; 0 selects 1 (forward) or 1/N (inverse).
 *   counts    device tfft_ft_counts, required unless ft_mode is TFFT_FT_OFF.
 * N must be 2^k or 3*2^k within the sizes the library supports
 * (tfft_supported()).  batch = 0 is a no-op. */
int tfft_c2c(const void* x, void* y, long long N, long long batch, int dir, int precision,
             int ft_mode, double scale, tfft_ft_counts* counts, void* hip_stream);

/* Offline (unfused) two-side ABFT, the comparison baseline for the fused
 * kernels (Sec. 2.2 offline FT-FFT; Sec. 5.2): the same transform as
 * tfft_c2c with TFFT_FT_CORRECT, but the checksums come from kernels of their
 * own that read the batch again, as a library-based scheme computes them:
 * an input pass (a^T x_b, |x_b|^2 and the right-side sum of each group of 16
 * consecutive signals), the plain transform, the transform of the right-side
 * sums, an output pass (e^T y_b) with a per-signal check against the same
 * threshold as the fused kernels, and a fix that rebuilds a group's faulty
 * signal as W(X e) - sum of the others (Eq. 5; two faults in a group are
 * counted uncorrectable).  counts (device) is required; detected, rebuilt,
 * uncorrectable and last_signal are updated.  Allocates a workspace per
 * (device, stream) of about (2 + 1/16) x the batch (grow-only, like the
 * two-pass workspace; a captured call that would allocate returns
 * TFFT_ECAPTURE).  An armed injection hits the plain transform. */
int tfft_c2c_offline(const void* x, void* y, long long N, long long batch, int dir, int precision,
                     double scale, tfft_ft_counts* counts, void* hip_stream);

/* The transform without ABFT at four levels of the stepwise study of the
 * transform itself (Sec. 5.1, versions v0..v3): single precision, N a power
 * of two, out of place (x and y must not overlap; TFFT_EINVAL otherwise).
 *   level 0  one kernel launch per radix-2 stage, each reading and writing
 *            global memory (log2 N launches, a library workspace for the
 *            intermediate);
 *   level 1  one launch, every radix-2 stage exchanged through LDS
 *            (N <= 8192, TFFT_EUNSUPPORTED beyond);
 *   level 2  the library's default route and plans (radix-16 stages, no
 *            tuning table);
 *   level 3  the tuned route (the tuning table's plain-mode entry), as
 *            tfft_c2c with TFFT_FT_OFF.
 * dir as for tfft_c2c; the inverse is scaled by 1/N.  A measurement aid:
 * all levels compute the same transform. */
int tfft_c2c_stepwise(const void* x, void* y, long long N, long long batch, int dir, int level,
                      void* hip_stream);

/* Size of the static device scratch buffer of tfft_c2c_noalloc (bytes). */
#define TFFT_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform, arguments, results and errors as tfft_c2c, but the call never
 * allocates.  The intermediate of a two-pass length lives in a static device
 * array of TFFT_NOALLOC_SCRATCH_BYTES (64 MiB) per device, held from the
 * first call on that device until the process ends; the transform runs over
 * chunks of signals that fit it.  Limits and errors, beyond tfft_c2c's:
 *   - TFFT_ESCRATCH when one signal (N * 8 bytes in fp32, N * 16 in fp64)
 *     is larger than the scratch buffer; any batch is accepted;
 *   - TFFT_ENOTPREPARED when the tables of (N, precision, ft_mode) were not
 *     built beforehand: call tfft_prepare(N, 0, precision, ft_mode, NULL)
 *     once first (that call allocates);
 *   - launches are never timed by tfft_profile.
 * Every call on one device shares that device's scratch array, whose
 * contents persist between calls (each call writes the intermediate before
 * reading it, so nothing needs clearing); calls that overlap in time on one
 * device (different streams, or host threads) race on it and must be ordered
 * by the caller. */
int tfft_c2c_noalloc(const void* x, void* y, long long N, long long batch, int dir, int precision,
                     int ft_mode, double scale, tfft_ft_counts* counts, void* hip_stream);

/* Build (and cache) the tables of length N for ABFT mode ft_mode and, when
 * batch > 0 and N runs as two passes, reserve the two-pass workspace that
 * tfft_c2c of up to `batch` signals on hip_stream will use.  Host call,
 * allocates, must not be made while hip_stream is being captured.  Call it
 * before capturing tfft_c2c into a graph: a captured call that finds its
 * tables or its workspace missing returns TFFT_ECAPTURE.
 * Workspace: one per (device, stream), owned by the library, grown when a
 * larger call needs it and never freed while the library is loaded, so a
 * graph captured earlier keeps a valid buffer; calls on one stream share it
 * (stream order serialises them), calls on different streams do not.
 * TFFT_EINVAL for N < 1, batch < 0 or an unknown enum; TFFT_EUNSUPPORTED for
 * a length without a compiled route; TFFT_ENOMEM when allocation fails. */
int tfft_prepare(long long N, long long batch, int precision, int ft_mode, void* hip_stream);

/* ---- Ragged batches: signals of mixed lengths in one call ----
 * The transform of each signal is that of tfft_c2c (Sec. 2.2), with the same
 * ABFT protection (Sec. 4), and per-signal results are bit-identical between
 * the two execution modes.  Signals are packed back to back in list order:
 * signal i occupies elements [sum_{j<i} sizes[j], sum_{j<=i} sizes[j]).
 *   TFFT_RAGGED_PERSISTENT  one persistent launch: workgroups take work items
 *                           (a group of signals of one length, or one tile of
 *                           a column / row pass) from a device queue; a row
 *                           pass waits on per-group counters for its column
 *                           pass.  Queue and counters reset themselves, so the
 *                           launch can be captured once and replayed.
 *   TFFT_RAGGED_PER_SIZE    one launch per length and pass, same kernel
 *                           bodies (the comparison baseline). */
typedef struct tfft_ragged_plan_s* tfft_ragged_plan;
enum { TFFT_RAGGED_PERSISTENT = 0, TFFT_RAGGED_PER_SIZE = 1 };

/* 1 if a signal of length N can be part of a ragged batch: TFFT_FP32 only,
 * N = 2^k for 6 <= k <= 17 or N = 3*2^k for 6 <= k <= 16. */
int tfft_ragged_supported(long long N, int precision);

/* Build a plan for `count` signals of lengths sizes_host[0..count) (HOST
 * array).  Allocates device memory owned by the plan: per-signal offset
 * tables, the work queue, the pass counters and a workspace of
 * sum(two-pass lengths) elements for column-pass results.  Call outside
 * stream capture.  TFFT_EUNSUPPORTED if a length has no ragged route or the
 * precision is not TFFT_FP32; *plan is NULL on error. */
int tfft_ragged_plan_create(tfft_ragged_plan* plan, const long long* sizes_host, long long count,
                            int precision);

/* Release a plan (after its launches have completed). */
int tfft_ragged_plan_destroy(tfft_ragged_plan plan);

/* Up to n values: [0] signals, [1] total elements, [2] work items,
 * [3] classes (lengths x passes), [4] workspace elements, [5] persistent
 * grid, [6] workspace batches and [7] window (elements per half; 0 when the
 * workspace is flat); [8] persistent launches of this plan in which a wait
 * gave up (sticky; each such launch also adds 1 to counts->sched_errors) and
 * [9] the queue's next-item counter (0 between launches); [8] and [9] are
 * read from the device with a synchronising copy when n > 8. */
int tfft_ragged_plan_info(tfft_ragged_plan plan, long long* info, int n);

/* Schedule of plans created from now on.  window_elems > 0: the persistent
 * launch streams the two-pass signals through a workspace ring of two halves
 * of window_elems elements (batches of whole checksum groups; a column pass
 * reuses a half once the row passes of the batch before last have read it),
 * so the intermediate can stay in the 256 MB on-die cache; 0 (default): one
 * workspace slot per signal, all column passes queued first.  item_elems > 0
 * sets the elements per work item (default 32768); 0 keeps it.  waves: 3
 * (default) holds the ABFT kernels to three workgroups per CU (a few values
 * spill; measured faster); 0 lets the compiler size their registers (two
 * workgroups per CU).  Per-size launches are unaffected. */
int tfft_ragged_set_schedule(long long window_elems, long long item_elems, int waves);

/* Test hook for the persistent launch's bounded waits: every row-pass (and
 * windowed column-pass) wait gives up after max_polls polls (0 restores the
 * default of 2^20) and needs `extra` more finished items than exist, so with
 * extra > 0 each wait reaches its bound: the launch still drains, reports the
 * failure (counts->sched_errors, plan info [8]) and resets its counters so
 * the next launch is correct.  Applies to launches made from now on. */
int tfft_ragged_test_wait(unsigned max_polls, unsigned extra);

/* Execute a plan.
 *   x, y        device buffers of total elements (complex64); x == y only
 *               with ft_mode below TFFT_FT_CORRECT (correction re-reads the
 *               inputs); partial overlap is not allowed.
 *   dir         TFFT_FORWARD or TFFT_INVERSE.
 *   unit_scale  0: outputs scaled by 1 (forward) or 1/N (inverse, per
 *               signal); 1: no scaling (the adjoint).
 *   mode        TFFT_RAGGED_PERSISTENT or TFFT_RAGGED_PER_SIZE.
 *   ft_mode     as in tfft_c2c; counts required unless TFFT_FT_OFF.
 * Allocates nothing and never synchronises, so it may be captured into a
 * hipGraph.  Launches of one plan share its queue and workspace and must not
 * overlap in time (same stream, or ordered). */
int tfft_c2c_ragged(tfft_ragged_plan plan, const void* x, void* y, int dir, int unit_scale,
                    int mode, int ft_mode, tfft_ft_counts* counts, void* hip_stream);

/* 1 if N (and precision) has a compiled kernel, else 0. */
int tfft_supported(long long N, int precision);

/* Test hook (Sec. 5.3 injection protocol; Sec. 2.2 fault model, a fault in
 * a compute unit that propagates through the later stages): arm a
 * single-bit flip for the NEXT tfft_c2c or tfft_c2c_ragged call only.
 *   signal     index of the signal in the call (ragged: index in the list).
 *   element    position of the value hit, in the numbering of the chosen
 *              pass: for a single-pass length, the position k < N in the
 *              sequence the chosen stage produces (after the last stage:
 *              output element k); for a two-pass length N = N1 * N2 (see
 *              tfft_route_info), in the column pass k * N2 + n2 (column n2,
 *              position k of its N1-point sequence; after the last stage the
 *              intermediate value of row k), in the row pass n1 + N1 * k (row
 *              n1, position k of its N2-point sequence; after the last stage
 *              output element n1 + N1 * k); for a three-pass length N = N1 *
 *              N2 * N3 (M = N2 * N3), where the value is stored within the
 *              signal: pass 0 k1 * M + m (column m), pass 1 k1 * M + k2 * N3
 *              + n3 (row k1, column n3, position k2), pass 2 the output
 *              element k1 + N1 * (k2 + N2 * k3) (row k1 of pair k2, position
 *              k3); after an earlier stage, the position the stage's
 *              sequence holds there.
 *   part       0: real part, 1: imaginary part.
 *   bit        bit of the IEEE binary32 (0..31) or binary64 (0..63) value.
 *   precision  TFFT_FP32 or TFFT_FP64; must match the call.
 *   pass       -1: the last pass; 0: the single pass or the column pass;
 *              1: the row pass (three passes: the second column pass); 2:
 *              the third pass of a three-pass length.
 *   stage      -1: after the last radix stage (an output value of the pass,
 *              before its checksum and store); s >= 0: after radix stage s,
 *              on the value held between stage s and s + 1.
 * The flip happens in registers inside the kernel.  The call returns
 * TFFT_EINVAL when the injection does not fit it (signal, element, pass or
 * stage out of range, other precision); arming returns TFFT_EINVAL for a
 * field out of range. */
typedef struct {
    long long signal, element;
    int part, bit, precision, pass, stage;
    int two;            /* 1: flip the same value of signal2 as well (two faults
                           in one call; signal2 != signal, and in a ragged
                           batch of the same length); 0: one fault */
    long long signal2;
} tfft_inject_desc;
int tfft_inject_arm_desc(const tfft_inject_desc* desc);

/* The same flip of an output value of the last pass (pass -1, stage -1). */
int tfft_inject_arm(long long signal, long long element, int part, int bit, int precision);
int tfft_inject_disarm(void);

/* Override the plan choices for (N, precision): transactions per slot T
 * (1..32) and the detection threshold factor kappa (> 0); pass 0 to keep a
 * value.  Used by the autotuner and by tests. */
int tfft_set_tuning(long long N, int precision, int T, double kappa);

/* Detection granularity for (N, precision) in every ABFT mode.
 *   0  once per group of T transactions (Sec. 4.3 multi-transaction
 *      threadblock ABFT): one reduction of D0 = sum_b (q_b - p_b) and of the
 *      location code D1 = sum_b (b+1)(q_b - p_b) per group, threshold from
 *      the group's input energy, faulty signal b* = D1/D0 - 1;
 *   1  per transaction (Sec. 4.1, delayed batched correction): each
 *      signal's q_b - p_b is checked against a threshold from its own input
 *      energy; a faulty signal is noted and repaired at the end of the group
 *      from the right-side sums of the transactions before the next faulty
 *      one (or of the whole group), oldest first.  A group then holds at most
 *      as many transactions as the plan's lanes per slot and wave (up to 16);
 *      a larger T is reduced to that.
 * Defaults: 1 for TFFT_FP32 (a per-signal threshold keeps an undetected
 * flip below the fp32 tolerance at any T), 0 for TFFT_FP64. */
int tfft_set_granularity(long long N, int precision, int gran);
int tfft_get_tuning(long long N, int precision, int* T, double* kappa);

/* Lengths above the single-pass limit run as a column pass and a row pass
 * (three passes: two intermediates) over chunks of signals whose
 * intermediate (chunk_bytes, default 128 MiB, at least one signal) lives in
 * a library workspace.  Sets the chunk size for (N, precision); 0 keeps the
 * current value. */
int tfft_set_chunk(long long N, int precision, long long chunk_bytes);

/* Routes.  A length runs as one single-pass kernel, as a column pass of
 * length n1 followed by a row pass of length N/n1 (the multi-pass
 * decomposition of Sec. 3.1), or as three passes N = n1 * n2 * n3 (the
 * three launches Sec. 3.3 gives lengths beyond 2^22): a column pass of n1
 * over the M = n2 * n3 columns, a column pass of n2 over the n3 columns of
 * each row of M with the twiddle w_N^{k1 m} applied at its load, and a row
 * pass of n3 with the twiddle w_M^{k2 n3} whose store transposes to the
 * output order k1 + n1 * (k2 + n2 * k3); up to N = 2^29 in single
 * precision.  Each pass takes one of the compiled plan variants of its
 * length (tile width).  A route is coded as
 *     code = n1 | va << 32 | vb << 40 | log2(n2) << 48
 * with n1 = 1 for a single pass of plan variant va; n1 > 1 and no n2 for a
 * column pass of variant va and a row pass of variant vb; n1 > 1 and n2 for
 * three passes, first column pass variant va and last row pass variant vb.  Code 0 is the default
 * policy (single pass when built, else the most balanced two-pass split,
 * else the three-pass split with the smallest largest length, variants 0).
 * The passes of three-pass routes check groups of one signal (T = 1).
 * tfft_routes writes up to cap codes built for (N, precision, ft_mode) and
 * returns how many exist.  tfft_set_route fixes the route of (N, precision)
 * in every ABFT mode (TFFT_EUNSUPPORTED if not built).  tfft_get_route
 * reports the route tfft_c2c would take now in ft_mode (never code 0).
 * tfft_set_tuning / tfft_set_chunk also apply to every mode; the tuning
 * table may set each mode apart. */
int tfft_routes(long long N, int precision, int ft_mode, long long* codes, int cap);

/* The route tfft_c2c takes now for (N, precision, ft_mode): up to n values
 * [0] passes (1, 2 or 3), [1] N1 (column-pass length; N for a single pass),
 * [2] N2 (length of pass 1; 1 for a single pass), [3] radix stages of pass
 * 0, [4] radix stages of pass 1 (0 for a single pass), [5] transactions per
 * checksum group T as launched, [6] detection granularity as launched (see
 * tfft_set_granularity; 0 without ABFT), [7] and [8] sub-signals per
 * workgroup of pass 0 and pass 1 (0 for a single pass), [9] N3 (length of
 * pass 2; 1 below three passes), [10] radix stages and [11] sub-signals per
 * workgroup of pass 2 (0 below three passes).  A launch of
 * directly addressed signals with G workgroups of s sub-signals forms G s
 * groups: transaction b of group g transforms signal g + b G s (single pass;
 * for a two-pass chunk, signal g + b * groups, each tile of a group taking
 * the same signals).  TFFT_EUNSUPPORTED for a length without a route. */
int tfft_route_info(long long N, int precision, int ft_mode, long long* info, int n);
int tfft_set_route(long long N, int precision, long long code);
int tfft_get_route(long long N, int precision, int ft_mode, long long* code);

/* Load a tuning table (JSON, as written by the autotuner):
 *   {"entries": [{"precision": "fp32" | "fp64", "N": n, "ft_mode": f,
 *                 "split_n1": s, "variant_a": va, "variant_b": vb,
 *                 "split_n2": n2 (three passes; absent or 0: two),
 *                 "T": t, "kappa": k, "chunk_bytes": b, ...}, ...]}
 * Each entry sets the fields it names for (N, precision) in ABFT mode f, or
 * in every mode when ft_mode is absent; other keys are ignored.  An optional
 * top-level "ragged": {"item_elems": n, "waves": 0 | 3} sets the schedule
 * of ragged plans created afterwards (as tfft_ragged_set_schedule).  All
 * entries are checked before any is applied.  Returns the number of entries
 * applied, or TFFT_EINVAL (unreadable file, malformed JSON or value out of
 * range) / TFFT_EUNSUPPORTED (a route not built). */
int tfft_load_tuning(const char* path);

/* Calibration of the detection threshold (Sec. 5.3 ROC protocol): while on,
 * every ABFT call also records in counts->calib the largest ratio
 * |D0| / tau over its fault-free groups, as the bits of an IEEE double
 * (atomic max; the caller zeroes it).  D0 is the left-side checksum
 * difference and tau the threshold.  Off by default; costs one atomic per
 * group. */
int tfft_calibration(int on);

/* Per-launch timing for benchmarks: while on, every kernel launch made by
 * tfft_c2c outside stream capture is bracketed by a pair of HIP events on its
 * stream.  tfft_profile_read synchronises on them, writes one text line per
 * kernel "precision kind Ns ft launches total_ms algorithmic_bytes" into buf
 * (host memory of buflen bytes), clears the log and returns the text length;
 * with buf == NULL it returns the size needed instead.  kind is single,
 * colpass, rowpass, ragged, colpass3 or rowpass3; algorithmic bytes count
 * each launch's input read and output write once.  Three more fields follow
 * on each line: the plan variant, E (elements per lane) and the width (sub-
 * signals per workgroup of a tile, waves per workgroup of a single pass), so
 * variants of one length are reported apart. */
int tfft_profile(int on);
int tfft_profile_read(char* buf, long long buflen);

/* Restrict the per-launch timing above to the launches of one kernel:
 * precision (TFFT_FP32 / TFFT_FP64), kind (0 single, 1 colpass, 2 rowpass,
 * 3 ragged persistent, 4 colpass3, 5 rowpass3: the second and third pass of
 * a three-pass length), sub-length Ns, ABFT mode ft and plan variant; -1 in a field
 * matches any value (all -1, the default, times every launch).  Events cost
 * the stream a few microseconds per launch, so a benchmark that times one
 * kernel live brackets only that kernel's launches.  Returns TFFT_EINVAL
 * for a value out of range. */
int tfft_profile_only(int precision, int kind, int Ns, int ft, int variant);

const char* tfft_strerror(int status);
int tfft_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TFFT_H */
