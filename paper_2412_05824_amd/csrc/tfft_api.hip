// tfft_api.hip -- host runtime behind the C ABI declared in include/tfft.h.
//
// Plans come from the compiled kernel registry.  Twiddle tables and the ABFT
// left vector e^T W are built here in long double, rounded once to the kernel
// precision, uploaded at prepare time and cached for the process.  Lengths
// above the single-pass limit run as a column pass and a row pass
// (N = N1 * N2, TurboFFT Sec. 3.1 kernel level), over chunks of signals so
// the intermediate stays in the on-package cache and the workspace is bounded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <cstdio>
#include <cstdlib>
#include <tuple>
#include <vector>

#include "tfft.h"
#include "tfft_offline.hpp"
#include "tfft_ragged.hpp"
#include "tfft_workspace.hpp"

using namespace tfft;

// Intermediate of two-pass transforms made through tfft_c2c_noalloc: one copy
// per device, held from the first such call on that device until the process
// ends, shared by every such call on that device.
static __device__ __align__(256) unsigned char scratch[TFFT_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return TFFT_EHIP;
}

// exp(-2 pi i num / den) with num reduced exactly modulo den and the angle
// folded into [0, pi/4] by the symmetries of sine and cosine.
void cis_neg(long long num, long long den, long double* re, long double* im) {
    const long double pi = 3.141592653589793238462643383279502884L;
    long long m = num % den;
    if (m < 0) m += den;
    bool neg = false;
    if (2 * m > den) { m = den - m; neg = true; }          // angle -> 2 pi - angle
    long double c, s;
    const long long q = 8 * m;
    if (q <= den) {
        long double a = 2.0L * pi * (long double)m / (long double)den;
        c = cosl(a); s = sinl(a);
    } else if (q <= 2 * den) {
        long double a = pi * (long double)(den - 4 * m) / (2.0L * (long double)den);
        c = sinl(a); s = cosl(a);
    } else if (q <= 3 * den) {
        long double a = pi * (long double)(4 * m - den) / (2.0L * (long double)den);
        c = -sinl(a); s = cosl(a);
    } else {
        long double a = pi * (long double)(den - 2 * m) / (long double)den;
        c = -cosl(a); s = sinl(a);
    }
    // exp(-i angle) = c - i s; the mirrored angle flips the sine
    *re = c;
    *im = neg ? s : -s;
}

struct SubTables {
    void* tw = nullptr;
    void* left = nullptr;
    void* cot = nullptr;             // cotangent form of the left vector (single passes)
    long double c2[2] = {0, 0};      // its factor (1 - w_M^N) / 2
};
struct PassTwiddle { void* hi = nullptr; void* lo = nullptr; int bits = 0; };

struct Tuning {
    int T;
    double kappa;
    long long chunk_bytes;
    long long route;      // route code (see route_for): 0 the default policy
    int gran;             // 0 detection once per group (location code), 1 per transaction
};

std::mutex g_mu;
std::vector<KernelEntry>* g_entries = nullptr;
std::map<std::tuple<int, int, int, int, int>, const KernelEntry*> g_by_key;   // (prec, kind, Ns, ft, variant)
std::map<std::pair<int, int>, const KernelEntry*> g_ragged_by_key;      // (ragged plan id, ft)
std::map<std::tuple<int, int, int, long long, int>, SubTables> g_sub;    // (prec, Ns, device, radices, single-pass lanes)
std::map<std::tuple<int, long long, int>, PassTwiddle> g_pass;           // (prec, N, device)
struct DeviceAlloc {
    bool operator()(void** p, size_t bytes) const {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) { g_last_hip = (int)e; *p = nullptr; return false; }
        return true;
    }
};
WorkspacePool<DeviceAlloc> g_ws{DeviceAlloc{}};                          // (device, stream)
WorkspacePool<DeviceAlloc> g_ws_off{DeviceAlloc{}};                      // offline ABFT, (device, stream)
std::map<std::tuple<int, long long, int>, void*> g_left_full;            // (prec, N, device): e^T W of N
std::map<std::tuple<int, long long, int>, Tuning> g_tuning;   // (prec, N, ft mode 0..2)

struct Inject {
    bool armed = false;
    long long signal = -1, element = 0;
    long long signal2 = -1;   // a second signal hit the same way (-1: none)
    int part = 0, bit = 0, precision = 0;
    int pass = -1;    // -1 last pass, 0 first (single or column pass), 1 row pass (three passes: 1, 2)
    int stage = -1;   // -1 after the last radix stage, else after stage `stage`
} g_inj;

// kernel-side injection fields of a launch that is pass `pass` (0 or 1) of a
// route with `passes` passes, of a plan with `stages` radix stages
template <class R> void arm_launch(KCall<R>& k, const Inject& inj, int pass, int passes, int stages) {
    k.inj_signal = -1;
    k.inj_signal2 = -1;
    if (!inj.armed) return;
    const int want = inj.pass < 0 ? passes - 1 : inj.pass;
    if (want != pass) return;
    k.inj_signal = inj.signal;
    k.inj_signal2 = inj.signal2;
    k.inj_elem = inj.element;
    k.inj_part = inj.part;
    k.inj_bit = inj.bit;
    k.inj_stage = inj.stage < 0 ? stages - 1 : inj.stage;
}

// an armed injection fits a route of passes first (, second (, third)):
// its pass exists and so does its stage
bool inject_fits(const Inject& inj, const KernelEntry* first, const KernelEntry* second,
                 const KernelEntry* third = nullptr) {
    if (!inj.armed) return true;
    const KernelEntry* e[3] = {first, second, third};
    const int passes = third ? 3 : (second ? 2 : 1);
    if (inj.pass >= passes || inj.pass < -1) return false;
    const KernelEntry* p = e[inj.pass < 0 ? passes - 1 : inj.pass];
    return inj.stage < p->n_stages && inj.stage >= -1;
}

bool g_stats = false;   // calibration mode: kernels record max |D0| / tau

// Optional per-launch timing: a HIP event pair around every kernel launch, on
// the launch stream, with the launch's algorithmic bytes (input + output).
struct LaunchRec {
    const KernelEntry* e;
    hipEvent_t start, stop;
    double bytes;
};
bool g_prof = false;
int g_prof_sel[5] = {-1, -1, -1, -1, -1};   // precision, kind, Ns, ft, variant of the timed kernel; -1: any
std::vector<LaunchRec> g_prof_log;
bool prof_selected(const KernelEntry& e) {
    const int v[5] = {e.precision, e.kind, e.Ns, e.ft, e.variant};
    for (int i = 0; i < 5; ++i)
        if (g_prof_sel[i] >= 0 && g_prof_sel[i] != v[i]) return false;
    return true;
}
std::string g_prof_text;   // aggregated, not yet read

void ensure_registry() {
    if (g_entries) return;
    g_entries = new std::vector<KernelEntry>();
    register_fp32_single(*g_entries);
    register_fp32_tiles(*g_entries);
    register_fp64_single(*g_entries);
    register_fp64_tiles(*g_entries);
    register_fp32_three(*g_entries);
    register_fp32_ragged_single(*g_entries);
    register_fp32_ragged_tiles(*g_entries);
    for (const KernelEntry& e : *g_entries) {
        if (e.ragged_id >= 0) g_ragged_by_key[std::make_pair(e.ragged_id, e.ft)] = &e;
        else g_by_key[std::make_tuple(e.precision, e.kind, e.Ns, e.ft, e.variant)] = &e;
    }
}

const KernelEntry* find_entry(int precision, int kind, long long Ns, int ft, int variant = 0) {
    if (Ns > (1 << 30) || variant < 0) return nullptr;
    auto it = g_by_key.find(std::make_tuple(precision, kind, (int)Ns, ft, variant));
    return it == g_by_key.end() ? nullptr : it->second;
}

// How a length is executed: one single-pass kernel, a column pass of
// length N1 and a row pass of length N2, or three passes N = N1 N2 N3
// (Sec. 3.3: three launches beyond 2^22): a column pass of N1 over the
// M = N2 N3 columns, a column pass of N2 over the N3 columns of each row
// (b, k1) with the outer twiddle w_N^{k1 m} at its load, and a row pass of
// N3 over each (b, k2) with the twiddle w_M^{k2 n3} that stores the output
// transposed, k1 + N1 (k2 + N2 k3).
struct Route {
    const KernelEntry* single = nullptr;
    const KernelEntry* col = nullptr;
    const KernelEntry* row = nullptr;    // two passes
    const KernelEntry* col3 = nullptr;   // three passes: second and third
    const KernelEntry* row3 = nullptr;
    long long N1 = 0, N2 = 0, N3 = 0;
    int passes() const { return single ? 1 : (row3 ? 3 : 2); }
    // entry of pass i
    const KernelEntry* pass(int i) const {
        if (single) return i == 0 ? single : nullptr;
        if (i == 0) return col;
        if (row3) return i == 1 ? col3 : (i == 2 ? row3 : nullptr);
        return i == 1 ? row : nullptr;
    }
};

// Route codes: n1 | va << 32 | vb << 40 | lg2(n2) << 48.  n1 = 1: single
// pass, plan variant va; n1 > 1 with no n2: column pass of n1 points
// (variant va), then row pass of N/n1 (variant vb); n1 > 1 with n2: the
// three passes N = n1 n2 (N / (n1 n2)), first column pass variant va, last
// row pass variant vb; code 0: the
// default policy (single pass when built, else the most balanced two-pass
// split, else the most balanced three-pass split, variants 0).
constexpr long long route_code(long long n1, int va, int vb, int lg_n2 = 0) {
    return n1 | ((long long)va << 32) | ((long long)vb << 40) | ((long long)lg_n2 << 48);
}
inline long long route_n1(long long code) { return code & 0xffffffffLL; }
inline int route_va(long long code) { return (int)((code >> 32) & 0xff); }
inline int route_vb(long long code) { return (int)((code >> 40) & 0xff); }
inline int route_lg_n2(long long code) { return (int)((code >> 48) & 0x3f); }

// a two-pass split N = n1 * n2 with compiled column and row kernels whose
// tiles divide the other length
bool split_ok(int precision, long long N, int ft, long long n1, int va = 0, int vb = 0) {
    if (n1 < 2 || N % n1) return false;
    const long long n2 = N / n1;
    const KernelEntry* c = find_entry(precision, kColPass, n1, ft, va);
    const KernelEntry* w = find_entry(precision, kRowPass, n2, ft, vb);
    return c && w && n2 % c->slots_per_block == 0 && n1 % w->slots_per_block == 0;
}

// Three passes reach N = 2^29 at most: every lane's byte offset within one
// transaction's span then stays below 2^32 (the buffer addressing range).
constexpr long long kMaxThreePassBytes = 1ll << 32;

// a three-pass split N = n1 n2 n3 with compiled kernels whose tiles divide
// the lengths they walk: M = n2 n3 columns of pass 1, n3 columns of pass 2,
// n1 rows of pass 3
bool split3_ok(int precision, long long N, int ft, long long n1, long long n2, int va = 0, int vb = 0) {
    if (n1 < 2 || n2 < 2 || N % (n1 * n2)) return false;
    const size_t S = precision == TFFT_FP32 ? 8 : 16;
    if ((double)N * (double)S > (double)kMaxThreePassBytes) return false;
    const long long n3 = N / (n1 * n2);
    const KernelEntry* a = find_entry(precision, kColPass, n1, ft, va);
    const KernelEntry* b = find_entry(precision, kColPass3, n2, ft, 0);
    const KernelEntry* c = find_entry(precision, kRowPass3, n3, ft, vb);
    return a && b && c && (n2 * n3) % a->slots_per_block == 0 && n3 % b->slots_per_block == 0 &&
           n1 % c->slots_per_block == 0;
}

int lg2(long long v) {
    int l = 0;
    while ((1ll << (l + 1)) <= v) ++l;
    return l;
}

bool route_for(int precision, long long N, int ft, Route* r, long long code = 0) {
    *r = Route{};
    if (code < 0 || (code >> 54) != 0) return false;
    const long long n1c = route_n1(code);
    const int va = route_va(code), vb = route_vb(code), lgn2 = route_lg_n2(code);
    if (code == 0 || n1c == 1) {
        if (lgn2 != 0) return false;
        if ((r->single = find_entry(precision, kSingle, N, ft, va))) return true;
        if (code != 0) return false;
    }
    long long n1 = 0, n2 = 0;
    if (code != 0) {
        if (lgn2 != 0) {
            if (!split3_ok(precision, N, ft, n1c, 1ll << lgn2, va, vb)) return false;
            n2 = 1ll << lgn2;
        } else if (!split_ok(precision, N, ft, n1c, va, vb)) {
            return false;
        }
        n1 = n1c;
    } else {
        // balanced split N = N1 * N2 with N1 <= N2
        for (long long c = 2; c * c <= N; c <<= 1)
            if (split_ok(precision, N, ft, c)) n1 = c;
        if (!n1) {
            // the three-pass split with the smallest largest length
            long long best = 0;
            for (long long a = 2; a < N; a <<= 1)
                for (long long b = 2; a * b < N; b <<= 1) {
                    if (!split3_ok(precision, N, ft, a, b)) continue;
                    const long long m = std::max(std::max(a, b), N / (a * b));
                    if (!best || m < best || (m == best && a > n1)) { best = m; n1 = a; n2 = b; }
                }
            if (!n1) return false;
        }
    }
    r->N1 = n1;
    if (n2) {
        r->N2 = n2;
        r->N3 = N / (n1 * n2);
        r->col = find_entry(precision, kColPass, n1, ft, code ? va : 0);
        r->col3 = find_entry(precision, kColPass3, n2, ft, 0);
        r->row3 = find_entry(precision, kRowPass3, r->N3, ft, code ? vb : 0);
        return true;
    }
    r->N2 = N / n1;
    r->col = find_entry(precision, kColPass, r->N1, ft, code ? va : 0);
    r->row = find_entry(precision, kRowPass, r->N2, ft, code ? vb : 0);
    return true;
}

// the route's code (what route_for reproduces it from)
long long code_of(const Route& r) {
    if (r.single) return route_code(1, r.single->variant, 0);
    if (r.row3) return route_code(r.N1, r.col->variant, r.row3->variant, lg2(r.N2));
    return route_code(r.N1, r.col->variant, r.row->variant);
}

Tuning default_tuning(int precision, long long N) {
    // Groups of T signals share one checksum reduction (Sec. 4.3).  Checked
    // once per group, an undetected flip just under the group's threshold
    // perturbs one signal by about kappa * u * sqrt(T log2 Ns) of its norm,
    // which in fp32 exceeds the 2e-6 tolerance unless T is 1 or 2; checked
    // per transaction (Sec. 4.1), each signal has its own threshold and T
    // only sets how many transactions share the right-side sums.  fp32
    // therefore checks per transaction, fp64 (ample margin) per group with
    // the location code.
    (void)N;
    Tuning t{};
    t.chunk_bytes = 128ll << 20;
    t.route = 0;
    if (precision == TFFT_FP32) {
        t.kappa = 8.0;
        t.T = 4;
        t.gran = 1;
    } else {
        t.kappa = 16.0;
        t.T = 8;
        t.gran = 0;
    }
    return t;
}

// The tuning a launch of plans pa (and pb, the row pass) really uses: no
// granularity without ABFT, and per-transaction checking limited to the
// transactions whose partials a plan keeps (the same T for both passes, so
// their signal groups coincide).
Tuning effective(const Tuning& tu, int ft, const KernelEntry* pa, const KernelEntry* pb = nullptr) {
    Tuning t = tu;
    if (ft == TFFT_FT_OFF) t.gran = 0;
    if (t.gran) {
        if (pa && t.T > pa->tx_max) t.T = pa->tx_max;
        if (pb && t.T > pb->tx_max) t.T = pb->tx_max;
        if (t.T < 1) t.T = 1;
    }
    return t;
}

// the tuning a route really uses.  The passes of a three-pass transform
// run groups of one signal: their signals are different units (signals,
// rows (b, k1), pairs (b, k2)), and a correction then needs the outer
// twiddle of one signal only.
Tuning effective(const Tuning& tu, int ft, const Route& rt) {
    if (rt.single) return effective(tu, ft, rt.single);
    if (!rt.row3) return effective(tu, ft, rt.col, rt.row);
    Tuning t = effective(tu, ft, rt.col, rt.col3);
    t.T = 1;
    return t;
}

// tuning of (precision, N) for an ABFT mode (the in-place correcting
// variant shares the correcting mode's entry)
Tuning get_tuning(int precision, long long N, int ft = TFFT_FT_CORRECT) {
    if (ft > TFFT_FT_CORRECT) ft = TFFT_FT_CORRECT;
    auto it = g_tuning.find(std::make_tuple(precision, N, ft));
    // detection without an entry of its own follows the correcting mode
    // (same kernels up to the correction path)
    if (it == g_tuning.end() && ft == TFFT_FT_DETECT)
        it = g_tuning.find(std::make_tuple(precision, N, (int)TFFT_FT_CORRECT));
    return it == g_tuning.end() ? default_tuning(precision, N) : it->second;
}

// apply fn to the tuning of (precision, N) in every ABFT mode
template <class F> void update_tuning(int precision, long long N, F fn) {
    for (int ft = 0; ft <= TFFT_FT_CORRECT; ++ft) {
        Tuning tu = get_tuning(precision, N, ft);
        fn(tu);
        g_tuning[std::make_tuple(precision, N, ft)] = tu;
    }
}

template <class R> void put(std::vector<R>& v, long double re, long double im) {
    v.push_back((R)re);
    v.push_back((R)im);
}

template <class R> int upload(const std::vector<R>& h, void** d) {
    hipError_t err = hipMalloc(d, h.size() * sizeof(R));
    if (err != hipSuccess) { g_last_hip = (int)err; *d = nullptr; return TFFT_ENOMEM; }
    err = hipMemcpy(*d, h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err);
    return TFFT_OK;
}

// a = e^T W of length N: a_n = (1 - w_M^N) / (1 - w_M w_N^n), w_M = exp(-2 pi i / M)
template <class R> int build_left(long long N, void** out) {
    const long long M = (N % 3 == 0) ? 5 : 3;
    std::vector<R> left;
    long double nr, ni;
    cis_neg(N, M, &nr, &ni);
    const long double num_re = 1.0L - nr, num_im = -ni;
    for (long long n = 0; n < N; ++n) {
        long double wr, wi;   // w_M w_N^n = exp(-2 pi i (N + M n) / (M N))
        cis_neg(N + M * n, M * N, &wr, &wi);
        const long double dr = 1.0L - wr, di = -wi;
        const long double den = dr * dr + di * di;
        put(left, (num_re * dr + num_im * di) / den, (num_im * dr - num_re * di) / den);
    }
    return upload(left, out);
}

// The left vector in cotangent form.  With w_M w_N^n = exp(-i theta_n),
// theta_n = 2 pi (N + M n) / (M N), 1 / (1 - exp(-i theta)) = (1 - i cot(theta / 2)) / 2,
// so a_n = c2 (1 - i cot(theta_n / 2)) with c2 = (1 - w_M^N) / 2: one real value
// per element.  Stored for lanes t < P holding elements t + P r (r < E), in
// 16-byte runs of G = 16 / sizeof(R) consecutive r: value (t, r) at
// ((r / G) P + t) G + r % G.
template <class R> int build_cot(long long N, int P, int E, SubTables* out) {
    const long long M = (N % 3 == 0) ? 5 : 3;
    const int G = 16 / (int)sizeof(R);
    if (E % G != 0 || (long long)P * E != N) return TFFT_EINVAL;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<R> cot((size_t)P * (size_t)E);
    for (int r = 0; r < E; ++r)
        for (int t = 0; t < P; ++t) {
            const long long n = t + (long long)P * r;
            // theta / 2 = pi k / (M N), k = (N + M n) mod (M N), never 0 (M does not divide N)
            const long long k = (N + M * n) % (M * N);
            const long double h = pi * (long double)k / (long double)(M * N);
            cot[((size_t)(r / G) * P + t) * G + r % G] = (R)(cosl(h) / sinl(h));
        }
    long double wr, wi;
    cis_neg(N, M, &wr, &wi);
    out->c2[0] = (1.0L - wr) / 2.0L;
    out->c2[1] = -wi / 2.0L;
    return upload(cot, &out->cot);
}

// stage tables w_{L R}^{j k} (k < L, j < R per stage) and a = e^T W
template <class R> int build_sub(const KernelEntry& e, SubTables* out) {
    const long long N = e.Ns;
    std::vector<R> tw;
    long long L = 1;
    for (int s = 0; s < e.n_stages; ++s) {
        const long long Rr = e.radices[s];
        for (long long k = 0; k < L; ++k)
            for (long long j = 0; j < Rr; ++j) {
                long double c, sn;
                cis_neg(j * k, L * Rr, &c, &sn);
                put(tw, c, sn);
            }
        L *= Rr;
    }
    int rc = upload(tw, &out->tw);
    if (rc != TFFT_OK) return rc;
    rc = build_left<R>(N, &out->left);
    // single passes: the cotangent form too, so that every mode of the plan
    // (those that read it and those that do not) shares one set of tables;
    // its layout needs whole 16-byte runs per lane (the kernels that read it
    // have them)
    if (rc != TFFT_OK || e.kind != kSingle || e.E % (16 / (int)sizeof(R)) != 0) return rc;
    return build_cot<R>(N, e.P, e.E, out);
}

// two-level table: w_N^m = hi[m >> bits] * lo[m & (2^bits - 1)]
template <class R> int build_pass(long long N, PassTwiddle* out) {
    int lg = 0;
    while ((1ll << (lg + 1)) <= N) ++lg;
    const int bits = (lg + 1) / 2;
    const long long nlo = 1ll << bits;
    const long long nhi = (N + nlo - 1) / nlo;
    std::vector<R> hi, lo;
    for (long long i = 0; i < nhi; ++i) {
        long double c, s;
        cis_neg(i * nlo, N, &c, &s);
        put(hi, c, s);
    }
    for (long long i = 0; i < nlo; ++i) {
        long double c, s;
        cis_neg(i, N, &c, &s);
        put(lo, c, s);
    }
    out->bits = bits;
    int rc = upload(hi, &out->hi);
    if (rc != TFFT_OK) return rc;
    return upload(lo, &out->lo);
}

int current_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Cached resources; built unless the stream is being captured.  Caller holds g_mu.
long long radix_signature(const KernelEntry& e) {
    long long sig = 0;   // radices <= 16, at most 14 stages: 17^14 < 2^63
    for (int s = 0; s < e.n_stages; ++s) sig = sig * 17 + e.radices[s];
    return sig;
}

int get_sub(const KernelEntry& e, bool may_alloc, SubTables** out) {
    auto key = std::make_tuple(e.precision, e.Ns, current_device(), radix_signature(e), e.kind == kSingle ? e.P : 0);
    auto it = g_sub.find(key);
    if (it != g_sub.end()) { *out = &it->second; return TFFT_OK; }
    if (!may_alloc) return TFFT_ECAPTURE;
    SubTables t;
    int rc = e.precision == TFFT_FP32 ? build_sub<float>(e, &t) : build_sub<double>(e, &t);
    if (rc != TFFT_OK) return rc;
    if (e.cot && !t.cot) return TFFT_EINVAL;   // a kernel that reads the cotangent table needs it
    *out = &(g_sub[key] = t);
    return TFFT_OK;
}

int get_pass(int precision, long long N, bool may_alloc, PassTwiddle** out) {
    auto key = std::make_tuple(precision, N, current_device());
    auto it = g_pass.find(key);
    if (it != g_pass.end()) { *out = &it->second; return TFFT_OK; }
    if (!may_alloc) return TFFT_ECAPTURE;
    PassTwiddle p;
    int rc = precision == TFFT_FP32 ? build_pass<float>(N, &p) : build_pass<double>(N, &p);
    if (rc != TFFT_OK) return rc;
    *out = &(g_pass[key] = p);
    return TFFT_OK;
}

// Thread-level ABFT table of a precision: for each radix R of 2, 4, 8, 16
// (at offset 2 (R - 2)), a = e^T W_R then a1 = e1^T W_R, e_k = w_3^k and
// e1_k = (k + 1) w_3^k, w = exp(-2 pi i / .), computed in long double.
template <class R> int build_thread_table(void** out) {
    std::vector<R> t;
    for (int Rr : {2, 4, 8, 16}) {
        for (int weighted = 0; weighted < 2; ++weighted)
            for (int n = 0; n < Rr; ++n) {
                long double re = 0, im = 0;
                for (int k = 0; k < Rr; ++k) {
                    long double c1, s1, c2, s2;
                    cis_neg(k % 3, 3, &c1, &s1);              // w_3^k
                    cis_neg((long long)k * n % Rr, Rr, &c2, &s2);   // w_R^{kn}
                    const long double w = weighted ? (long double)(k + 1) : 1.0L;
                    re += w * (c1 * c2 - s1 * s2);
                    im += w * (c1 * s2 + s1 * c2);
                }
                put(t, re, im);
            }
    }
    return upload(t, out);
}

std::map<std::tuple<int, int>, void*> g_thr;   // (precision, device) -> thread-level table

int get_thread_table(int precision, bool may_alloc, void** out) {
    auto key = std::make_tuple(precision, current_device());
    auto it = g_thr.find(key);
    if (it != g_thr.end()) { *out = it->second; return TFFT_OK; }
    if (!may_alloc) return TFFT_ECAPTURE;
    void* d = nullptr;
    int rc = precision == TFFT_FP32 ? build_thread_table<float>(&d) : build_thread_table<double>(&d);
    if (rc != TFFT_OK) return rc;
    *out = g_thr[key] = d;
    return TFFT_OK;
}

int get_workspace(size_t bytes, hipStream_t stream, bool may_alloc, void** out) {
    switch (g_ws.get(current_device(), stream, bytes, may_alloc, out)) {
        case WsResult::kOk: return TFFT_OK;
        case WsResult::kWouldAllocate: return TFFT_ECAPTURE;
        default: return TFFT_ENOMEM;
    }
}

// signals per chunk of a two-pass transform: the tuned chunk in whole
// signals, at least one, at most the batch
long long chunk_signals(long long N, long long batch, size_t elem_bytes, const Tuning& tu) {
    long long chunk = tu.chunk_bytes / (long long)((size_t)N * elem_bytes);
    if (chunk < 1) chunk = 1;
    if (chunk > batch) chunk = batch;
    return chunk;
}

template <class V> struct Launch {
    using R = typename RealOf<V>::type;
    KArgs<V> a{};
    const KernelEntry* e = nullptr;
};

template <class V>
void fill_common(KArgs<V>& a, const KernelEntry& e, const SubTables& st, const Tuning& tu,
                 tfft_ft_counts* counts) {
    using R = typename RealOf<V>::type;
    a.tw = static_cast<const V*>(st.tw);
    a.left = static_cast<const V*>(st.left);
    a.cot = static_cast<const R*>(st.cot);
    a.cot_c2 = V{(R)st.c2[0], (R)st.c2[1]};
    a.T = tu.T;
    a.gran = tu.gran;
    const double u = e.precision == TFFT_FP32 ? 0x1p-24 : 0x1p-53;
    const double Ns = (double)e.Ns;
    // rounding steps per element behind the checked difference: log2 Ns
    // for the butterflies, and three more where a pass multiplies its input
    // by an inter-pass twiddle (the twiddle, a product of two table values,
    // then its products with the value and with the left vector)
    const bool tw = e.kind == kRowPass || e.kind == kColPass3 || e.kind == kRowPass3;
    const double steps = std::log2(Ns) + (tw ? 3.0 : 0.0);
    a.tau_coef = (R)(tu.kappa * u * std::sqrt(Ns * steps));
    a.cap = e.precision == TFFT_FP32 ? (R)0x1p64 : (R)0x1p512;
    a.counts = reinterpret_cast<FtCounts*>(counts);
    a.inj_signal = -1;
    a.inj_signal2 = -1;
    a.stats = g_stats ? 1 : 0;
}

template <class V> int run(const KernelEntry& e, const void* x, void* y, const KArgs<V>& a,
                           long long grid, hipStream_t stream, bool timed = true) {
    if (grid <= 0) return TFFT_OK;
    if (grid > 0x7fffffffLL) return TFFT_EUNSUPPORTED;
    LaunchRec rec{};
    const bool prof = timed && g_prof && !capturing(stream) && prof_selected(e);
    if (prof) {
        rec.e = &e;
        // a three-pass row pass's signals are pairs (b, k2) of N / N2 elements
        const double len = e.kind == kRowPass3 ? (double)a.N / (double)a.p3_n2 : (double)a.N;
        rec.bytes = 2.0 * (double)a.batch * len * (double)sizeof(V);
        if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.stop) != hipSuccess)
            return hip_fail(hipGetLastError());
        (void)hipEventRecord(rec.start, stream);
    }
    hipError_t err = e.launch(x, y, &a, grid, stream);
    if (prof) {
        (void)hipEventRecord(rec.stop, stream);
        g_prof_log.push_back(rec);
    }
    return err == hipSuccess ? TFFT_OK : hip_fail(err);
}

// Where a two-pass transform keeps its intermediate: the library workspace of
// (device, stream), or a fixed caller-side buffer of `cap` bytes (the
// no-allocation entry point), in which case chunks shrink to fit it and no
// launch is timed.
struct WsSource {
    void* fixed = nullptr;
    size_t cap = 0;
};

// Injection target of pass 1 or 2 of a three-pass transform.  The caller
// numbers element e by where that pass stores it within the signal: pass 1
// row k1 = e / M, element e mod M (k2 N3 + n3); pass 2 the transposed
// output e = k1 + N1 (k2 + N2 k3), which lies in pair (b, k2) at position
// k1 + N1 k3 of the pass's row numbering.
template <class R> void arm_three(KCall<R>& k, const Inject& inj, int pass, const Route& rt) {
    arm_launch(k, inj, pass, 3, rt.pass(pass)->n_stages);
    if (k.inj_signal < 0 || pass == 0) return;
    const long long M = rt.N2 * rt.N3, e = inj.element;
    auto sub = [&](long long b) {
        if (b < 0) return b;
        return pass == 1 ? b * rt.N1 + e / M : b * rt.N2 + (e / rt.N1) % rt.N2;
    };
    k.inj_signal = sub(inj.signal);
    k.inj_signal2 = sub(inj.signal2);
    k.inj_elem = pass == 1 ? e % M : e % rt.N1 + rt.N1 * (e / (rt.N1 * rt.N2));
}

// Three passes over chunks of whole signals, each out of place: x -> ws0
// (column pass of N1), ws0 -> ws1 (column pass of N2 within each row), ws1
// -> y (row pass of N3, transposed store).  Two intermediates of a chunk
// each, so every pass keeps its input intact for the correction's re-read.
template <class V>
int transform3(const Route& rt, const void* x, void* y, long long N, long long batch, int conj,
               double scale, tfft_ft_counts* counts, const Tuning& tu, const Inject& inj,
               hipStream_t stream, bool may_alloc, const WsSource& wsrc) {
    using R = typename RealOf<V>::type;
    const int precision = sizeof(R) == 4 ? TFFT_FP32 : TFFT_FP64;
    const long long N1 = rt.N1, N2 = rt.N2, N3 = rt.N3, M = N2 * N3;
    SubTables *sa = nullptr, *sb = nullptr, *sc = nullptr;
    PassTwiddle *ptN = nullptr, *ptM = nullptr;
    int rc = get_sub(*rt.col, may_alloc, &sa);
    if (rc == TFFT_OK) rc = get_sub(*rt.col3, may_alloc, &sb);
    if (rc == TFFT_OK) rc = get_sub(*rt.row3, may_alloc, &sc);
    if (rc == TFFT_OK) rc = get_pass(precision, N, may_alloc, &ptN);
    if (rc == TFFT_OK) rc = get_pass(precision, M, may_alloc, &ptM);
    if (rc != TFFT_OK) return rc;
    const size_t sig_bytes = (size_t)N * sizeof(V);
    long long chunk = chunk_signals(N, batch, sizeof(V), tu);
    void* ws = nullptr;
    const bool timed = wsrc.fixed == nullptr;
    if (wsrc.fixed) {
        if (2 * sig_bytes > wsrc.cap) return TFFT_ESCRATCH;
        chunk = std::min(chunk, (long long)(wsrc.cap / (2 * sig_bytes)));
        ws = wsrc.fixed;
    } else {
        rc = get_workspace(2 * (size_t)chunk * sig_bytes, stream, may_alloc, &ws);
        if (rc != TFFT_OK) return rc;
    }
    char* ws0 = static_cast<char*>(ws);
    char* ws1 = ws0 + (size_t)chunk * sig_bytes;

    KArgs<V> A{}, B{}, C{};
    fill_common(A, *rt.col, *sa, tu, counts);
    fill_common(B, *rt.col3, *sb, tu, counts);
    fill_common(C, *rt.row3, *sc, tu, counts);
    for (KArgs<V>* k : {&A, &B, &C}) k->x_intact = 1;
    // pass A: columns m of each signal, stride M
    A.N = N; A.N1 = (int)N1; A.N2 = (int)M;
    A.tiles = (int)(M / rt.col->slots_per_block);
    A.conj_in = conj; A.conj_out = 0; A.scale = (R)1;
    // pass B: rows (b, k1) of length M, columns n3 at stride N3
    B.N = M; B.N1 = (int)N2; B.N2 = (int)N3;
    B.p3_n1 = (int)N1;
    B.tiles = (int)(N3 / rt.col3->slots_per_block);
    B.tw_hi = static_cast<const V*>(ptN->hi);
    B.tw_lo = static_cast<const V*>(ptN->lo);
    B.tw_bits = ptN->bits;
    B.conj_in = 0; B.conj_out = 0; B.scale = (R)1;
    // pass C: pairs (b, k2), rows k1 at stride M, transposed store
    C.N = N; C.N1 = (int)N1; C.N2 = (int)N3;
    C.p3_n2 = (int)N2; C.p3_M = M;
    C.tiles = (int)(N1 / rt.row3->slots_per_block);
    C.tw_hi = static_cast<const V*>(ptM->hi);
    C.tw_lo = static_cast<const V*>(ptM->lo);
    C.tw_bits = ptM->bits;
    C.conj_in = 0; C.conj_out = conj; C.scale = (R)scale;

    const char* xb = static_cast<const char*>(x);
    char* yb = static_cast<char*>(y);
    for (long long c0 = 0; c0 < batch; c0 += chunk) {
        const long long cnt = (batch - c0 < chunk) ? batch - c0 : chunk;
        A.batch = cnt;
        A.sig_base = c0;
        B.batch = cnt * N1;
        B.sig_base = c0 * N1;
        C.batch = cnt * N2;
        C.sig_base = c0 * N2;
        arm_three(A, inj, 0, rt);
        arm_three(B, inj, 1, rt);
        arm_three(C, inj, 2, rt);
        const bool hit = (inj.signal >= c0 && inj.signal < c0 + cnt) ||
                         (inj.signal2 >= c0 && inj.signal2 < c0 + cnt);
        if (!hit)
            for (KArgs<V>* k : {&A, &B, &C}) k->inj_signal = k->inj_signal2 = -1;
        rc = run<V>(*rt.col, xb + (size_t)c0 * sig_bytes, ws0, A, A.batch * A.tiles, stream, timed);
        if (rc == TFFT_OK) rc = run<V>(*rt.col3, ws0, ws1, B, B.batch * B.tiles, stream, timed);
        if (rc == TFFT_OK)
            rc = run<V>(*rt.row3, ws1, yb + (size_t)c0 * sig_bytes, C, C.batch * C.tiles, stream, timed);
        if (rc != TFFT_OK) return rc;
    }
    return TFFT_OK;
}

template <class V>
int transform(const Route& rt, const void* x, void* y, long long N, long long batch, int dir,
              double scale, tfft_ft_counts* counts, const Tuning& tu_in, const Inject& inj,
              hipStream_t stream, bool may_alloc, const WsSource& wsrc = WsSource{}) {
    using R = typename RealOf<V>::type;
    const Tuning tu = effective(tu_in, rt.pass(0)->ft, rt);
    const int precision = sizeof(R) == 4 ? TFFT_FP32 : TFFT_FP64;
    const int conj = dir == TFFT_INVERSE ? 1 : 0;
    if (rt.single) {
        SubTables* st = nullptr;
        int rc = get_sub(*rt.single, may_alloc, &st);
        if (rc != TFFT_OK) return rc;
        KArgs<V> a{};
        fill_common(a, *rt.single, *st, tu, counts);
        a.batch = batch;
        a.N = N;
        a.conj_in = a.conj_out = conj;
        a.scale = (R)scale;
        a.sig_base = 0;
        a.x_intact = x != y ? 1 : 0;
        if (rt.single->ft == 4) {
            void* tt = nullptr;
            rc = get_thread_table(precision, may_alloc, &tt);
            if (rc != TFFT_OK) return rc;
            a.thr_tab = static_cast<const V*>(tt);
            a.thr_ku = (R)(tu.kappa * (precision == TFFT_FP32 ? 0x1p-24 : 0x1p-53));
        }
        arm_launch(a, inj, 0, 1, rt.single->n_stages);
        const long long per_block = (long long)rt.single->slots_per_block * tu.T;
        return run<V>(*rt.single, x, y, a, (batch + per_block - 1) / per_block, stream,
                      wsrc.fixed == nullptr);
    }
    if (rt.row3)
        return transform3<V>(rt, x, y, N, batch, conj, scale, counts, tu, inj, stream, may_alloc, wsrc);
    // two passes over chunks of signals
    SubTables *sa = nullptr, *sb = nullptr;
    PassTwiddle* pt = nullptr;
    int rc = get_sub(*rt.col, may_alloc, &sa);
    if (rc == TFFT_OK) rc = get_sub(*rt.row, may_alloc, &sb);
    if (rc == TFFT_OK) rc = get_pass(precision, N, may_alloc, &pt);
    if (rc != TFFT_OK) return rc;
    const size_t sig_bytes = (size_t)N * sizeof(V);
    long long chunk = chunk_signals(N, batch, sizeof(V), tu);
    void* ws = nullptr;
    const bool timed = wsrc.fixed == nullptr;
    if (wsrc.fixed) {
        if (sig_bytes > wsrc.cap) return TFFT_ESCRATCH;
        chunk = std::min(chunk, (long long)(wsrc.cap / sig_bytes));
        ws = wsrc.fixed;
    } else {
        rc = get_workspace((size_t)chunk * sig_bytes, stream, may_alloc, &ws);
        if (rc != TFFT_OK) return rc;
    }

    KArgs<V> A{}, B{};
    fill_common(A, *rt.col, *sa, tu, counts);
    fill_common(B, *rt.row, *sb, tu, counts);
    for (KArgs<V>* k : {&A, &B}) {
        k->N = N;
        k->N1 = (int)rt.N1;
        k->N2 = (int)rt.N2;
        k->x_intact = 1;   // pass A reads x (untouched until pass B of the chunk), pass B reads Z
    }
    A.conj_in = conj; A.conj_out = 0; A.scale = (R)1;
    B.conj_in = 0; B.conj_out = conj; B.scale = (R)scale;
    B.tw_hi = static_cast<const V*>(pt->hi);
    B.tw_lo = static_cast<const V*>(pt->lo);
    B.tw_bits = pt->bits;
    A.tiles = (int)(rt.N2 / rt.col->slots_per_block);
    B.tiles = (int)(rt.N1 / rt.row->slots_per_block);

    const char* xb = static_cast<const char*>(x);
    char* yb = static_cast<char*>(y);
    for (long long c0 = 0; c0 < batch; c0 += chunk) {
        const long long cnt = (batch - c0 < chunk) ? batch - c0 : chunk;
        A.batch = B.batch = cnt;
        A.sig_base = B.sig_base = c0;
        // global signal index: the kernels compare sig_base + s
        arm_launch(A, inj, 0, 2, rt.col->n_stages);
        arm_launch(B, inj, 1, 2, rt.row->n_stages);
        // a chunk holding neither target runs without the hook
        const bool hit = (inj.signal >= c0 && inj.signal < c0 + cnt) ||
                         (inj.signal2 >= c0 && inj.signal2 < c0 + cnt);
        if (!hit) A.inj_signal = B.inj_signal = A.inj_signal2 = B.inj_signal2 = -1;
        const long long groups = (cnt + tu.T - 1) / tu.T;
        rc = run<V>(*rt.col, xb + (size_t)c0 * sig_bytes, ws, A, groups * A.tiles, stream, timed);
        if (rc != TFFT_OK) return rc;
        rc = run<V>(*rt.row, ws, yb + (size_t)c0 * sig_bytes, B, groups * B.tiles, stream, timed);
        if (rc != TFFT_OK) return rc;
    }
    return TFFT_OK;
}


// ---------------------------------------------------------------------------
// Ragged batches: signals of mixed lengths packed back to back.
// ---------------------------------------------------------------------------

// route of one length through the ragged plan list
struct RRoute {
    const KernelEntry* single = nullptr;   // FT-0 entries; other modes share ids
    const KernelEntry* col = nullptr;
    const KernelEntry* row = nullptr;
    long long N1 = 0, N2 = 0;
};

const KernelEntry* ragged_entry(int id, int ft) {
    auto it = g_ragged_by_key.find(std::make_pair(id, ft));
    return it == g_ragged_by_key.end() ? nullptr : it->second;
}

const KernelEntry* ragged_find(int kind, long long Ns) {
    for (auto& kv : g_ragged_by_key)
        if (kv.first.second == 0 && kv.second->kind == kind && kv.second->Ns == Ns) return kv.second;
    return nullptr;
}

bool ragged_route(long long N, RRoute* r) {
    *r = RRoute{};
    if (N < 1 || N > (1 << 30)) return false;
    if ((r->single = ragged_find(kSingle, N))) return true;
    long long best = 0;
    for (long long n1 = 2; n1 * n1 <= N; ++n1) {
        if (N % n1) continue;
        const KernelEntry* c = ragged_find(kColPass, n1);
        const KernelEntry* w = ragged_find(kRowPass, N / n1);
        // whole tiles only: a column tile spans slots_per_block of the N / n1
        // columns, a row tile slots_per_block of the n1 rows
        if (c && w && (N / n1) % c->slots_per_block == 0 && n1 % w->slots_per_block == 0) best = n1;
    }
    if (!best) return false;
    r->N1 = best;
    r->N2 = N / best;
    r->col = ragged_find(kColPass, r->N1);
    r->row = ragged_find(kRowPass, r->N2);
    return true;
}

KernelEntry g_ragged_prof_entry[3];   // labels of the persistent launches in the profile
long long g_ragged_window = 0;        // workspace window of new plans (elements, 0: flat)
long long g_ragged_item = 32768;      // elements per work item of new plans
int g_ragged_waves = 3;               // persistent kernel register budget of new plans
unsigned g_ragged_max_polls = 0;      // test hook: bound of one wait (0: the default)
unsigned g_ragged_wait_extra = 0;     // test hook: added to what every wait needs

RaggedKernel ragged_kernel(int ft, int waves) {
    static RaggedKernel k[3][2];
    static bool done[3][2] = {};
    const int w = waves == 3 ? 1 : 0;
    if (!done[ft][w]) {
        k[ft][w] = ft == 0 ? ragged_kernel_ft0(waves) : ft == 1 ? ragged_kernel_ft1(waves) : ragged_kernel_ft2(waves);
        done[ft][w] = true;
    }
    return k[ft][w];
}

}  // namespace

struct tfft_ragged_plan_s {
    int device = 0;
    int precision = TFFT_FP32;
    long long count = 0, total = 0, ws_elems = 0;
    std::vector<long long> sizes;          // host copy, for argument checks
    std::vector<RClass> classes;           // host copy (per-size launches, queue order)
    long long n_items = 0;
    long long n_batches = 0;               // windowed workspace: batches of groups
    long long window = 0;                  // windowed workspace: elements per half (0: flat)
    int waves = 0;                         // persistent kernel variant (0 or 3)
    int cus = 0;
    void* buf = nullptr;                   // classes, items, desc, queue, counters, tables
    void* ws = nullptr;                    // column-pass results of the two-pass signals
    RaggedDesc* d_desc = nullptr;
    RQueue* d_queue = nullptr;
};

namespace {

int ragged_build(tfft_ragged_plan_s* P, const long long* sizes, long long count) {
    P->count = count;
    P->sizes.assign(sizes, sizes + count);
    std::vector<long long> xoff(count);
    long long tot = 0;
    for (long long i = 0; i < count; ++i) { xoff[i] = tot; tot += sizes[i]; }
    P->total = tot;

    // one entry per distinct length, longest first
    std::map<long long, std::vector<long long>, std::greater<long long>> by_len;
    for (long long i = 0; i < count; ++i) by_len[sizes[i]].push_back(i);
    struct Len {
        RRoute rt;
        std::vector<long long> ids;
        long long N = 0, groups = 0;
        Tuning tu{};
        int T = 1;
        size_t ids_at = 0, xoff_at = 0, wsflat_at = 0, wsring_at = 0;
        int k_single = 1, k_col = 1, k_row = 1;   // blocks per work item
        RClass single{}, col{}, row{};
        int ci_single = -1, ci_col = -1, ci_row = -1;
    };
    std::vector<Len> lens;
    for (auto& kv : by_len) {
        Len L;
        if (!ragged_route(kv.first, &L.rt)) return TFFT_EUNSUPPORTED;
        L.ids = kv.second;
        L.N = kv.first;
        // per-transaction checking: T within what every plan of the route
        // keeps (the FT-0 entries carry the same plan limits as the others)
        L.tu = L.rt.single ? effective(get_tuning(TFFT_FP32, L.N), TFFT_FT_CORRECT, L.rt.single)
                           : effective(get_tuning(TFFT_FP32, L.N), TFFT_FT_CORRECT, L.rt.col, L.rt.row);
        L.T = L.tu.T;
        L.groups = ((long long)L.ids.size() + L.T - 1) / L.T;
        lens.push_back(std::move(L));
    }
    // blocks per work item: about g_ragged_item elements, so that the queue
    // and descriptor traffic of an item is small next to its data; tile runs
    // stay inside one group of signals
    // ... but at least about four items per resident workgroup, so that a
    // small batch still spreads over the whole GPU
    hipDeviceProp_t prop{};
    hipError_t perr = hipGetDeviceProperties(&prop, P->device);
    if (perr != hipSuccess) return hip_fail(perr);
    P->cus = prop.multiProcessorCount;
    long long work = 0;   // element passes of the whole batch
    for (Len& L : lens) work += (long long)L.ids.size() * L.N * (L.rt.single ? 1 : 2);
    const long long resident =
        std::max(1ll, (long long)ragged_kernel(TFFT_FT_CORRECT, P->waves).blocks_per_cu * P->cus);
    const long long item_elems = std::max(1ll, std::min(g_ragged_item, work / (4 * resident)));
    auto per_item = [item_elems](const KernelEntry& e, int T, int tiles) {
        const long long per_block = (long long)e.slots_per_block * T * e.Ns;
        long long k = item_elems / per_block;
        if (k < 1) k = 1;
        if (tiles > 0) {
            if (k > tiles) k = tiles;
            while (tiles % k) --k;
        }
        return (int)k;
    };

    // host tables (int64): ids, x offsets, flat and ring workspace offsets
    std::vector<long long> tab;
    long long ws_flat = 0, groups_tot = 0, max_group = 0;
    for (Len& L : lens) {
        const long long n = (long long)L.ids.size();
        L.ids_at = tab.size();
        for (long long i : L.ids) tab.push_back(i);
        L.xoff_at = tab.size();
        for (long long i : L.ids) tab.push_back(xoff[i]);
        if (L.rt.single) {
            const KernelEntry& e = *L.rt.single;
            SubTables* st = nullptr;
            int rc = get_sub(e, true, &st);
            if (rc != TFFT_OK) return rc;
            RClass& c = L.single;
            fill_common(c.args, e, *st, L.tu, nullptr);
            c.args.batch = n;
            c.args.N = L.N;
            c.args.x_intact = 1;
            c.plan = e.ragged_id;
            c.final_pass = 1;
            const long long per_block = (long long)e.slots_per_block * L.T;
            c.nblocks = (int)((n + per_block - 1) / per_block);
            c.cnt_base = -1;
            L.k_single = per_item(e, L.T, 0);
            continue;
        }
        L.wsflat_at = tab.size();
        for (long long j = 0; j < n; ++j) { tab.push_back(ws_flat); ws_flat += L.N; }
        L.wsring_at = tab.size();
        tab.resize(tab.size() + (size_t)n, 0);   // filled below when windowed
        max_group = std::max(max_group, (long long)L.T * L.N);
        SubTables *sa = nullptr, *sb = nullptr;
        PassTwiddle* pt = nullptr;
        int rc = get_sub(*L.rt.col, true, &sa);
        if (rc == TFFT_OK) rc = get_sub(*L.rt.row, true, &sb);
        if (rc == TFFT_OK) rc = get_pass(TFFT_FP32, L.N, true, &pt);
        if (rc != TFFT_OK) return rc;
        RClass& A = L.col;
        RClass& B = L.row;
        fill_common(A.args, *L.rt.col, *sa, L.tu, nullptr);
        fill_common(B.args, *L.rt.row, *sb, L.tu, nullptr);
        for (RClass* k : {&A, &B}) {
            k->args.batch = n;
            k->args.N = L.N;
            k->args.N1 = (int)L.rt.N1;
            k->args.N2 = (int)L.rt.N2;
            k->args.x_intact = 1;
            k->cnt_base = (int)groups_tot;
        }
        B.args.tw_hi = static_cast<const float2*>(pt->hi);
        B.args.tw_lo = static_cast<const float2*>(pt->lo);
        B.args.tw_bits = pt->bits;
        A.args.tiles = A.tiles = (int)(L.rt.N2 / L.rt.col->slots_per_block);
        B.args.tiles = B.tiles = (int)(L.rt.N1 / L.rt.row->slots_per_block);
        A.plan = L.rt.col->ragged_id;
        B.plan = L.rt.row->ragged_id;
        A.dst_ws = 1;
        A.signal_after = 1;
        B.src_ws = 1;
        B.final_pass = 1;
        L.k_col = per_item(*L.rt.col, L.T, A.tiles);
        L.k_row = per_item(*L.rt.row, L.T, B.tiles);
        A.items_per_group = A.tiles / L.k_col;
        B.items_per_group = B.tiles / L.k_row;
        B.need = A.items_per_group;
        if (L.groups * A.tiles > 0x7fffffffLL || L.groups * B.tiles > 0x7fffffffLL) return TFFT_EUNSUPPORTED;
        A.nblocks = (int)(L.groups * A.tiles);
        B.nblocks = (int)(L.groups * B.tiles);
        groups_tot += L.groups;
    }

    // class order (also the per-size launch order): column passes, single
    // passes, row passes, each longest first
    std::vector<RClass> classes;
    for (Len& L : lens)
        if (!L.rt.single) { L.ci_col = (int)classes.size(); classes.push_back(L.col); }
    for (Len& L : lens)
        if (L.rt.single) { L.ci_single = (int)classes.size(); classes.push_back(L.single); }
    for (Len& L : lens)
        if (!L.rt.single) { L.ci_row = (int)classes.size(); classes.push_back(L.row); }

    // workspace window: batches of whole groups of at most W elements; batch
    // k uses half k % 2 of a 2W ring
    long long W = g_ragged_window;
    const bool windowed = W > 0 && ws_flat > 0;
    if (windowed && W < max_group) W = max_group;
    struct GroupRef { Len* L; long long g; };
    std::vector<std::vector<GroupRef>> batches;
    if (windowed) {
        long long fill = W;   // forces a first batch
        for (Len& L : lens) {
            if (L.rt.single) continue;
            const long long n = (long long)L.ids.size();
            for (long long g = 0; g < L.groups; ++g) {
                const long long s0 = g * L.T, s1 = std::min(n, s0 + L.T);
                const long long e = (s1 - s0) * L.N;
                if (fill + e > W) { batches.emplace_back(); fill = 0; }
                const long long base = (long long)((batches.size() - 1) % 2) * W + fill;
                for (long long j = s0; j < s1; ++j) tab[L.wsring_at + (size_t)j] = base + (j - s0) * L.N;
                fill += e;
                batches.back().push_back(GroupRef{&L, g});
            }
        }
    }
    P->n_batches = (long long)batches.size();

    // items (the queue order)
    std::vector<RItem> items;
    auto run = [&](int ci, long long b0, long long b1, int k, int batch, int wait_batch, int wait_need) {
        for (long long b = b0; b < b1; b += k)
            items.push_back(RItem{ci, (int)b, (int)std::min<long long>(k, b1 - b), batch, wait_batch,
                                  wait_need, 0, 0});
    };
    std::vector<int> rows_in_batch(batches.size(), 0);
    for (size_t k = 0; k < batches.size(); ++k)
        for (GroupRef& gr : batches[k]) rows_in_batch[k] += gr.L->row.items_per_group;
    auto col_items = [&](size_t k) {
        const int wb = k >= 2 ? (int)(k - 2) : -1;
        const int wn = k >= 2 ? rows_in_batch[k - 2] : 0;
        for (GroupRef& gr : batches[k]) {
            const long long t = gr.L->col.tiles;
            run(gr.L->ci_col, gr.g * t, (gr.g + 1) * t, gr.L->k_col, -1, wb, wn);
        }
    };
    auto row_items = [&](size_t k) {
        for (GroupRef& gr : batches[k]) {
            const long long t = gr.L->row.tiles;
            run(gr.L->ci_row, gr.g * t, (gr.g + 1) * t, gr.L->k_row, (int)k, -1, 0);
        }
    };
    if (windowed) {
        for (size_t k = 0; k < batches.size(); ++k) {
            col_items(k);
            if (k >= 1) row_items(k - 1);
        }
        if (!batches.empty()) row_items(batches.size() - 1);
        for (Len& L : lens)
            if (L.rt.single) run(L.ci_single, 0, L.single.nblocks, L.k_single, -1, -1, 0);
    } else {
        for (Len& L : lens)
            if (!L.rt.single) run(L.ci_col, 0, L.col.nblocks, L.k_col, -1, -1, 0);
        for (Len& L : lens)
            if (L.rt.single) run(L.ci_single, 0, L.single.nblocks, L.k_single, -1, -1, 0);
        for (Len& L : lens)
            if (!L.rt.single) run(L.ci_row, 0, L.row.nblocks, L.k_row, -1, -1, 0);
    }
    P->n_items = (long long)items.size();
    const long long ws_elems = std::max(ws_flat, windowed ? 2 * W : 0ll);
    P->ws_elems = ws_elems;
    P->window = windowed ? W : 0;

    // one device buffer: classes | items | desc | queue | cnt_a | cnt_b | cnt_r | tables
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t o_cls = 0;
    const size_t o_items = al(o_cls + classes.size() * sizeof(RClass));
    const size_t o_desc = al(o_items + items.size() * sizeof(RItem));
    const size_t o_q = al(o_desc + sizeof(RaggedDesc));
    const size_t o_ca = al(o_q + sizeof(RQueue));
    const size_t o_cb = al(o_ca + (size_t)groups_tot * sizeof(unsigned));
    const size_t o_cr = al(o_cb + (size_t)groups_tot * sizeof(unsigned));
    const size_t o_tab = al(o_cr + batches.size() * sizeof(unsigned));
    const size_t bytes = al(o_tab + tab.size() * sizeof(long long));
    hipError_t err = hipMalloc(&P->buf, bytes);
    if (err != hipSuccess) { g_last_hip = (int)err; P->buf = nullptr; return TFFT_ENOMEM; }
    if (ws_elems > 0) {
        err = hipMalloc(&P->ws, (size_t)ws_elems * sizeof(float2));
        if (err != hipSuccess) { g_last_hip = (int)err; P->ws = nullptr; return TFFT_ENOMEM; }
    }
    char* base = static_cast<char*>(P->buf);
    const long long* dtab = reinterpret_cast<const long long*>(base + o_tab);
    // host copies (per-size launches) use the flat workspace offsets, the
    // device copies (persistent launch) the ring offsets when windowed
    std::vector<RClass> dev_classes = classes;
    for (Len& L : lens) {
        if (L.rt.single) {
            for (std::vector<RClass>* v : {&classes, &dev_classes}) {
                RClass& c = (*v)[L.ci_single];
                c.args.id_tab = dtab + L.ids_at;
                c.args.in_tab = c.args.out_tab = dtab + L.xoff_at;
            }
            continue;
        }
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<RClass>& v = pass == 0 ? classes : dev_classes;
            const long long* ws = dtab + ((pass == 1 && windowed) ? L.wsring_at : L.wsflat_at);
            RClass& A = v[L.ci_col];
            RClass& B = v[L.ci_row];
            A.args.id_tab = B.args.id_tab = dtab + L.ids_at;
            A.args.in_tab = dtab + L.xoff_at;
            A.args.out_tab = ws;
            B.args.in_tab = ws;
            B.args.out_tab = dtab + L.xoff_at;
        }
    }
    P->classes = classes;
    RaggedDesc desc{};
    desc.classes = reinterpret_cast<const RClass*>(base + o_cls);
    desc.items = reinterpret_cast<const RItem*>(base + o_items);
    desc.n_items = P->n_items;
    desc.q = reinterpret_cast<RQueue*>(base + o_q);
    desc.cnt_a = reinterpret_cast<unsigned*>(base + o_ca);
    desc.cnt_b = reinterpret_cast<unsigned*>(base + o_cb);
    desc.cnt_r = reinterpret_cast<unsigned*>(base + o_cr);
    desc.n_batches = (long long)batches.size();
    desc.n_groups = groups_tot;
    desc.ws = static_cast<float2*>(P->ws);
    P->d_desc = reinterpret_cast<RaggedDesc*>(base + o_desc);
    P->d_queue = desc.q;

    std::vector<char> host(bytes, 0);
    memcpy(host.data() + o_cls, dev_classes.data(), dev_classes.size() * sizeof(RClass));
    memcpy(host.data() + o_items, items.data(), items.size() * sizeof(RItem));
    memcpy(host.data() + o_desc, &desc, sizeof(desc));
    memcpy(host.data() + o_tab, tab.data(), tab.size() * sizeof(long long));
    err = hipMemcpy(P->buf, host.data(), bytes, hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err);

    return TFFT_OK;
}

int ragged_exec(tfft_ragged_plan_s* P, const void* x, void* y, int dir, int unit_scale, int mode,
                int ft, tfft_ft_counts* counts, const Inject& inj, hipStream_t stream) {
    RaggedCall c{};
    c.x = static_cast<const float2*>(x);
    c.y = static_cast<float2*>(y);
    c.counts = reinterpret_cast<FtCounts*>(counts);
    c.inj_signal = inj.armed ? inj.signal : -1;
    c.inj_signal2 = inj.armed ? inj.signal2 : -1;
    c.inj_elem = inj.element;
    c.inj_part = inj.part;
    c.inj_bit = inj.bit;
    c.inj_pass = inj.pass;
    c.inj_stage = inj.stage;
    c.conj = dir == TFFT_INVERSE ? 1 : 0;
    c.unit_scale = unit_scale ? 1 : 0;
    c.stats = g_stats ? 1 : 0;
    c.max_polls = g_ragged_max_polls ? g_ragged_max_polls : kMaxPolls;
    c.wait_extra = g_ragged_wait_extra;
    if (P->n_items == 0) return TFFT_OK;
    if (mode == TFFT_RAGGED_PERSISTENT) {
        const RaggedKernel k = ragged_kernel(ft, P->waves);
        if (!k.launch || k.blocks_per_cu <= 0) return TFFT_EUNSUPPORTED;
        long long grid = (long long)k.blocks_per_cu * P->cus;
        if (grid > P->n_items) grid = P->n_items;
        LaunchRec rec{};
        KernelEntry& pe = g_ragged_prof_entry[ft];
        pe.precision = TFFT_FP32;
        pe.kind = 3;
        pe.Ns = 0;
        pe.ft = ft;
        const bool prof = g_prof && !capturing(stream) && prof_selected(pe);
        if (prof) {
            rec.e = &pe;
            rec.bytes = 2.0 * (double)P->total * (double)sizeof(float2);
            if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.stop) != hipSuccess)
                return hip_fail(hipGetLastError());
            (void)hipEventRecord(rec.start, stream);
        }
        hipError_t err = k.launch(c, P->d_desc, (int)grid, stream);
        if (prof) {
            (void)hipEventRecord(rec.stop, stream);
            g_prof_log.push_back(rec);
        }
        return err == hipSuccess ? TFFT_OK : hip_fail(err);
    }
    // one launch per class, in queue order (column passes, single, row passes)
    for (const RClass& cl : P->classes) {
        const KernelEntry* e = ragged_entry(cl.plan, ft);
        if (!e) return TFFT_EUNSUPPORTED;
        KArgs<float2> a = cl.args;
        a.conj_in = cl.src_ws ? 0 : c.conj;
        a.conj_out = cl.final_pass ? c.conj : 0;
        a.scale = (cl.final_pass && c.conj && !c.unit_scale) ? 1.0f / (float)a.N : 1.0f;
        a.counts = c.counts;
        a.stats = c.stats;
        {
            const int passes = (cl.src_ws || cl.dst_ws) ? 2 : 1;
            arm_launch(a, inj, cl.src_ws ? 1 : 0, passes, e->n_stages);
        }
        const void* src = cl.src_ws ? P->ws : x;
        void* dst = cl.dst_ws ? P->ws : y;
        int rc = run<float2>(*e, src, dst, a, cl.nblocks, stream);
        if (rc != TFFT_OK) return rc;
    }
    return TFFT_OK;
}


// ---------------------------------------------------------------------------
// Tuning table file (JSON): {"entries": [{"precision": "fp32" | "fp64" | 0 | 1,
// "N": n, "ft_mode": f, "split_n1": s, "variant_a": va, "variant_b": vb,
// "T": t, "kappa": k, "chunk_bytes": b, ...}, ...]}.  An entry without
// ft_mode applies to every ABFT mode.  Unknown keys are ignored; missing
// ones keep their current value.
// ---------------------------------------------------------------------------
struct JVal {
    enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const char* k) const {
        for (auto& kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const std::string& t;
    size_t i = 0;
    explicit JParser(const std::string& text) : t(text) {}
    void ws() { while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\r' || t[i] == '\t')) ++i; }
    bool lit(const char* w) {
        const size_t n = strlen(w);
        if (t.compare(i, n, w) != 0) return false;
        i += n;
        return true;
    }
    bool str(std::string* out) {
        if (i >= t.size() || t[i] != '"') return false;
        ++i;
        out->clear();
        while (i < t.size() && t[i] != '"') {
            char ch = t[i++];
            if (ch == '\\') {
                if (i >= t.size()) return false;
                const char e = t[i++];
                if (e == 'u') {   // keep ASCII only
                    if (i + 4 > t.size()) return false;
                    ch = (char)std::strtol(t.substr(i, 4).c_str(), nullptr, 16);
                    i += 4;
                } else {
                    ch = e == 'n' ? '\n' : e == 't' ? '\t' : e == 'r' ? '\r' : e == 'b' ? '\b' : e == 'f' ? '\f' : e;
                }
            }
            out->push_back(ch);
        }
        if (i >= t.size()) return false;
        ++i;
        return true;
    }
    bool value(JVal* v, int depth) {
        if (depth > 32) return false;
        ws();
        if (i >= t.size()) return false;
        const char c = t[i];
        if (c == '{') {
            ++i;
            v->kind = JVal::kObj;
            ws();
            if (i < t.size() && t[i] == '}') { ++i; return true; }
            for (;;) {
                ws();
                std::string k;
                if (!str(&k)) return false;
                ws();
                if (i >= t.size() || t[i] != ':') return false;
                ++i;
                JVal e;
                if (!value(&e, depth + 1)) return false;
                v->obj.emplace_back(std::move(k), std::move(e));
                ws();
                if (i < t.size() && t[i] == ',') { ++i; continue; }
                if (i < t.size() && t[i] == '}') { ++i; return true; }
                return false;
            }
        }
        if (c == '[') {
            ++i;
            v->kind = JVal::kArr;
            ws();
            if (i < t.size() && t[i] == ']') { ++i; return true; }
            for (;;) {
                JVal e;
                if (!value(&e, depth + 1)) return false;
                v->arr.push_back(std::move(e));
                ws();
                if (i < t.size() && t[i] == ',') { ++i; continue; }
                if (i < t.size() && t[i] == ']') { ++i; return true; }
                return false;
            }
        }
        if (c == '"') { v->kind = JVal::kStr; return str(&v->str); }
        if (lit("true")) { v->kind = JVal::kBool; v->num = 1; return true; }
        if (lit("false")) { v->kind = JVal::kBool; v->num = 0; return true; }
        if (lit("null")) { v->kind = JVal::kNull; return true; }
        char* end = nullptr;
        const double d = std::strtod(t.c_str() + i, &end);
        if (end == t.c_str() + i) return false;
        i = (size_t)(end - t.c_str());
        v->kind = JVal::kNum;
        v->num = d;
        return true;
    }
};

bool json_int(const JVal* v, long long* out) {
    if (!v || v->kind != JVal::kNum || v->num != std::floor(v->num)) return false;
    *out = (long long)v->num;
    return true;
}

bool is_pow2(long long n) { return n > 0 && (n & (n - 1)) == 0; }

int check_precision(int p) { return (p == TFFT_FP32 || p == TFFT_FP64) ? TFFT_OK : TFFT_EINVAL; }

}  // namespace

extern "C" {

const char* tfft_strerror(int status) {
    switch (status) {
        case TFFT_OK: return "ok";
        case TFFT_EINVAL: return "invalid argument";
        case TFFT_EUNSUPPORTED: return "unsupported size or mode";
        case TFFT_EALIGN: return "misaligned buffer";
        case TFFT_EHIP: return "HIP runtime error";
        case TFFT_ENOMEM: return "out of device memory";
        case TFFT_ECAPTURE: return "allocation needed during stream capture";
        case TFFT_ENOTPREPARED: return "tables not built: call tfft_prepare for this length first";
        case TFFT_ESCRATCH: return "one signal exceeds the no-allocation scratch buffer (64 MiB)";
        default: return "unknown status";
    }
}

int tfft_last_hip_error(void) { return g_last_hip; }

int tfft_supported(long long N, int precision) {
    if (check_precision(precision) != TFFT_OK || N < 1) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    Route r;
    return route_for(precision, N, 0, &r) ? 1 : 0;
}

int tfft_prepare(long long N, long long batch, int precision, int ft_mode, void* hip_stream) {
    if (N < 1 || batch < 0 || check_precision(precision) != TFFT_OK || ft_mode < 0 || ft_mode > 2)
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    const Tuning tu = get_tuning(precision, N, ft_mode);
    Route r;
    if (!route_for(precision, N, ft_mode, &r, tu.route)) return TFFT_EUNSUPPORTED;
    SubTables* st = nullptr;
    if (r.single) {
        int rc = get_sub(*r.single, true, &st);
        // the in-place correcting kernel shares the tables of its plan
        return rc;
    }
    int rc = TFFT_OK;
    for (int i = 0; i < r.passes() && rc == TFFT_OK; ++i) rc = get_sub(*r.pass(i), true, &st);
    PassTwiddle* pt = nullptr;
    if (rc == TFFT_OK) rc = get_pass(precision, N, true, &pt);
    if (rc == TFFT_OK && r.row3) rc = get_pass(precision, r.N2 * r.N3, true, &pt);
    if (rc == TFFT_OK && batch > 0) {
        const size_t S = precision == TFFT_FP32 ? 8 : 16;
        void* ws = nullptr;
        // three passes hold two intermediates of a chunk
        rc = get_workspace((size_t)(r.row3 ? 2 : 1) * (size_t)chunk_signals(N, batch, S, tu) * (size_t)N * S,
                           static_cast<hipStream_t>(hip_stream), true, &ws);
    }
    return rc;
}

int tfft_set_tuning(long long N, int precision, int T, double kappa) {
    if (N < 1 || check_precision(precision) != TFFT_OK || T < 0 || T > 32 || kappa < 0) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    update_tuning(precision, N, [&](Tuning& tu) {
        if (T > 0) tu.T = T;
        if (kappa > 0) tu.kappa = kappa;
    });
    return TFFT_OK;
}

int tfft_routes(long long N, int precision, int ft_mode, long long* codes, int cap) {
    if (N < 1 || check_precision(precision) != TFFT_OK || ft_mode < 0 || ft_mode > 2 || cap < 0 ||
        (cap > 0 && !codes))
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    int n = 0;
    auto put_route = [&](long long v) {
        if (n < cap) codes[n] = v;
        ++n;
    };
    for (int v = 0; v < 8; ++v)
        if (find_entry(precision, kSingle, N, ft_mode, v)) put_route(route_code(1, v, 0));
    for (long long c = 2; c < N; c <<= 1)
        for (int va = 0; va < 8; ++va)
            for (int vb = 0; vb < 8; ++vb)
                if (split_ok(precision, N, ft_mode, c, va, vb)) put_route(route_code(c, va, vb));
    for (long long c = 2; c < N; c <<= 1)
        for (long long b = 2; c * b < N; b <<= 1)
            for (int va = 0; va < 8; ++va)
                for (int vb = 0; vb < 8; ++vb)
                    if (split3_ok(precision, N, ft_mode, c, b, va, vb)) put_route(route_code(c, va, vb, lg2(b)));
    return n;
}

// route of (precision, N) in one ABFT mode (ft 0..2) or in all (ft < 0)
int set_route_locked(long long N, int precision, int ft, long long code) {
    Route r;
    for (int f = 0; f <= TFFT_FT_CORRECT; ++f)
        if ((ft < 0 || f == ft) && code != 0 && !route_for(precision, N, f, &r, code)) return TFFT_EUNSUPPORTED;
    for (int f = 0; f <= TFFT_FT_CORRECT; ++f) {
        if (ft >= 0 && f != ft) continue;
        Tuning tu = get_tuning(precision, N, f);
        tu.route = code;
        g_tuning[std::make_tuple(precision, N, f)] = tu;
    }
    return TFFT_OK;
}

int tfft_set_route(long long N, int precision, long long code) {
    if (N < 1 || check_precision(precision) != TFFT_OK || code < 0) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    return set_route_locked(N, precision, -1, code);
}

int tfft_route_info(long long N, int precision, int ft_mode, long long* info, int n) {
    if (!info || n < 1 || N < 1 || check_precision(precision) != TFFT_OK || ft_mode < 0 || ft_mode > 2)
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    const Tuning tu = get_tuning(precision, N, ft_mode);
    Route r;
    if (!route_for(precision, N, ft_mode, &r, tu.route)) return TFFT_EUNSUPPORTED;
    long long v[12] = {};
    const KernelEntry* p0 = r.pass(0);
    const KernelEntry* p1 = r.pass(1);
    const KernelEntry* p2 = r.pass(2);
    v[0] = r.passes();
    v[1] = r.single ? N : r.N1;
    v[2] = r.single ? 1 : r.N2;
    v[3] = p0->n_stages;
    v[4] = p1 ? p1->n_stages : 0;
    v[7] = p0->slots_per_block;
    v[8] = p1 ? p1->slots_per_block : 0;
    v[9] = r.row3 ? r.N3 : 1;
    v[10] = p2 ? p2->n_stages : 0;
    v[11] = p2 ? p2->slots_per_block : 0;
    const Tuning te = effective(tu, ft_mode, r);
    v[5] = te.T;
    v[6] = te.gran;
    for (int i = 0; i < n && i < 12; ++i) info[i] = v[i];
    return TFFT_OK;
}

int tfft_set_granularity(long long N, int precision, int gran) {
    if (N < 1 || check_precision(precision) != TFFT_OK || gran < 0 || gran > 1) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    update_tuning(precision, N, [&](Tuning& tu) { tu.gran = gran; });
    return TFFT_OK;
}

int tfft_get_route(long long N, int precision, int ft_mode, long long* code) {
    if (!code || N < 1 || check_precision(precision) != TFFT_OK || ft_mode < 0 || ft_mode > 2)
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    Route r;
    const long long c = get_tuning(precision, N, ft_mode).route;
    if (!route_for(precision, N, ft_mode, &r, c)) return TFFT_EUNSUPPORTED;
    *code = code_of(r);
    return TFFT_OK;
}

int tfft_load_tuning(const char* path) {
    if (!path) return TFFT_EINVAL;
    FILE* f = fopen(path, "rb");
    if (!f) return TFFT_EINVAL;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    JVal root;
    JParser jp(text);
    if (!jp.value(&root, 0) || root.kind != JVal::kObj) return TFFT_EINVAL;
    const JVal* entries = root.get("entries");
    if (!entries || entries->kind != JVal::kArr) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    // validate every entry before applying any
    std::vector<std::pair<std::tuple<int, long long, int>, Tuning>> pending;
    auto current = [&](int prec, long long N, int ft) {
        Tuning tu = get_tuning(prec, N, ft);
        for (auto& q : pending)
            if (q.first == std::make_tuple(prec, N, ft)) tu = q.second;
        return tu;
    };
    for (const JVal& e : entries->arr) {
        if (e.kind != JVal::kObj) return TFFT_EINVAL;
        const JVal* pv = e.get("precision");
        int prec = -1;
        if (pv && pv->kind == JVal::kStr) prec = pv->str == "fp32" ? TFFT_FP32 : pv->str == "fp64" ? TFFT_FP64 : -1;
        else if (pv && pv->kind == JVal::kNum) prec = (int)pv->num;
        long long N = 0;
        if (check_precision(prec) != TFFT_OK || !json_int(e.get("N"), &N) || N < 1) return TFFT_EINVAL;
        long long ftv = -1;   // absent: every mode
        if (e.get("ft_mode") && (!json_int(e.get("ft_mode"), &ftv) || ftv < 0 || ftv > 2)) return TFFT_EINVAL;
        for (int ft = 0; ft <= TFFT_FT_CORRECT; ++ft) {
            if (ftv >= 0 && ft != ftv) continue;
            Tuning tu = current(prec, N, ft);
            long long v = 0;
            if (e.get("split_n1")) {
                long long va = 0, vb = 0, n2 = 0;
                if (!json_int(e.get("split_n1"), &v) || v < 0 || v > 0xffffffffLL) return TFFT_EINVAL;
                if (e.get("variant_a") && (!json_int(e.get("variant_a"), &va) || va < 0 || va > 255)) return TFFT_EINVAL;
                if (e.get("variant_b") && (!json_int(e.get("variant_b"), &vb) || vb < 0 || vb > 255)) return TFFT_EINVAL;
                // three passes: the second length, a power of two
                if (e.get("split_n2") && (!json_int(e.get("split_n2"), &n2) || n2 < 0 || n2 > (1ll << 30) ||
                                          (n2 != 0 && (n2 < 2 || (n2 & (n2 - 1))))))
                    return TFFT_EINVAL;
                const long long code = v == 0 ? 0 : route_code(v, (int)va, (int)vb, n2 ? lg2(n2) : 0);
                Route r;
                if (code != 0 && !route_for(prec, N, ft, &r, code)) return TFFT_EUNSUPPORTED;
                tu.route = code;
            }
            if (e.get("T")) {
                if (!json_int(e.get("T"), &v) || v < 1 || v > 32) return TFFT_EINVAL;
                tu.T = (int)v;
            }
            if (e.get("gran")) {
                if (!json_int(e.get("gran"), &v) || v < 0 || v > 1) return TFFT_EINVAL;
                tu.gran = (int)v;
            }
            if (e.get("chunk_bytes")) {
                if (!json_int(e.get("chunk_bytes"), &v) || v < 1) return TFFT_EINVAL;
                tu.chunk_bytes = v;
            }
            if (const JVal* k = e.get("kappa")) {
                if (k->kind != JVal::kNum || !(k->num > 0)) return TFFT_EINVAL;
                tu.kappa = k->num;
            }
            bool found = false;
            for (auto& q : pending)
                if (q.first == std::make_tuple(prec, N, ft)) { q.second = tu; found = true; }
            if (!found) pending.emplace_back(std::make_tuple(prec, N, ft), tu);
        }
    }
    // the ragged schedule of plans created afterwards: elements per work item
    // and the ABFT kernels' register budget (waves 0 or 3)
    long long r_item = 0, r_waves = -1;
    if (const JVal* rg = root.get("ragged")) {
        if (rg->kind != JVal::kObj) return TFFT_EINVAL;
        if (rg->get("item_elems") && (!json_int(rg->get("item_elems"), &r_item) || r_item < 1 || r_item > (1ll << 30)))
            return TFFT_EINVAL;
        if (rg->get("waves") && (!json_int(rg->get("waves"), &r_waves) || (r_waves != 0 && r_waves != 3)))
            return TFFT_EINVAL;
    }
    for (auto& q : pending) g_tuning[q.first] = q.second;
    if (r_item > 0) g_ragged_item = r_item;
    if (r_waves >= 0) g_ragged_waves = (int)r_waves;
    return (int)entries->arr.size();
}

int tfft_get_tuning(long long N, int precision, int* T, double* kappa) {
    if (!T || !kappa || check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Tuning tu = get_tuning(precision, N, TFFT_FT_CORRECT);
    *T = tu.T;
    *kappa = tu.kappa;
    return TFFT_OK;
}

int tfft_set_chunk(long long N, int precision, long long chunk_bytes) {
    if (N < 1 || check_precision(precision) != TFFT_OK || chunk_bytes < 0) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    update_tuning(precision, N, [&](Tuning& tu) {
        if (chunk_bytes > 0) tu.chunk_bytes = chunk_bytes;
    });
    return TFFT_OK;
}

int tfft_profile(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof = on != 0;
    return TFFT_OK;
}

int tfft_profile_only(int precision, int kind, int Ns, int ft, int variant) {
    if (precision < -1 || precision > TFFT_FP64 || kind < -1 || kind > 5 || Ns < -1 || ft < -1 || ft > 3 ||
        variant < -1 || variant > 255)
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof_sel[0] = precision;
    g_prof_sel[1] = kind;
    g_prof_sel[2] = Ns;
    g_prof_sel[3] = ft;
    g_prof_sel[4] = variant;
    return TFFT_OK;
}

int tfft_profile_read(char* buf, long long buflen) {
    std::lock_guard<std::mutex> lk(g_mu);
    // aggregate the pending launches per kernel: launches, total ms, bytes
    struct Agg { long long n = 0; double ms = 0, bytes = 0; };
    // per plan: precision, kind, Ns, ft, variant, E, width (sub-signals of a
    // tile, waves of a single-pass workgroup)
    std::map<std::tuple<int, int, int, int, int, int, int>, Agg> agg;
    for (LaunchRec& r : g_prof_log) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            const int width = r.e->kind == kSingle ? r.e->threads / 64 : r.e->slots_per_block;
            Agg& g = agg[std::make_tuple(r.e->precision, r.e->kind, r.e->Ns, r.e->ft, r.e->variant, r.e->E, width)];
            g.n += 1;
            g.ms += ms;
            g.bytes += r.bytes;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof_log.clear();
    static const char* kinds[] = {"single", "colpass", "rowpass", "ragged", "colpass3", "rowpass3"};
    for (auto& kv : agg) {
        char line[256];
        snprintf(line, sizeof(line), "%s %s %d %d %lld %.6f %.1f %d %d %d\n",
                 std::get<0>(kv.first) == TFFT_FP32 ? "fp32" : "fp64", kinds[std::get<1>(kv.first)],
                 std::get<2>(kv.first), std::get<3>(kv.first), kv.second.n, kv.second.ms, kv.second.bytes,
                 std::get<4>(kv.first), std::get<5>(kv.first), std::get<6>(kv.first));
        g_prof_text += line;
    }
    if (!buf) return (int)g_prof_text.size() + 1;   // size query keeps the text
    if ((long long)g_prof_text.size() + 1 > buflen) return TFFT_EINVAL;
    memcpy(buf, g_prof_text.c_str(), g_prof_text.size() + 1);
    const int n = (int)g_prof_text.size();
    g_prof_text.clear();
    return n;
}

int tfft_calibration(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_stats = on != 0;
    return TFFT_OK;
}

int tfft_inject_arm_desc(const tfft_inject_desc* d) {
    if (!d) return TFFT_EINVAL;
    if (d->signal < 0 || d->element < 0 || (d->part != 0 && d->part != 1)) return TFFT_EINVAL;
    if (check_precision(d->precision) != TFFT_OK) return TFFT_EINVAL;
    const int width = d->precision == TFFT_FP32 ? 32 : 64;
    if (d->bit < 0 || d->bit >= width) return TFFT_EINVAL;
    if (d->pass < -1 || d->pass > 2 || d->stage < -1) return TFFT_EINVAL;
    if (d->two != 0 && (d->two != 1 || d->signal2 < 0 || d->signal2 == d->signal)) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_inj.armed = true;
    g_inj.signal = d->signal;
    g_inj.element = d->element;
    g_inj.part = d->part;
    g_inj.bit = d->bit;
    g_inj.precision = d->precision;
    g_inj.pass = d->pass;
    g_inj.stage = d->stage;
    g_inj.signal2 = d->two ? d->signal2 : -1;
    return TFFT_OK;
}

int tfft_inject_arm(long long signal, long long element, int part, int bit, int precision) {
    tfft_inject_desc d{};
    d.signal = signal;
    d.element = element;
    d.part = part;
    d.bit = bit;
    d.precision = precision;
    d.pass = -1;
    d.stage = -1;
    return tfft_inject_arm_desc(&d);
}

int tfft_inject_disarm(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_inj = Inject{};
    return TFFT_OK;
}

}  // extern "C"

namespace {

// Device address of `scratch` on each device, resolved once per device with
// that device current (the array's name in host code is only a stand-in for
// the symbol, not a device address).  Caller holds g_mu.
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_device(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return TFFT_EUNSUPPORTED;
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TFFT_OK;
}

// Argument checks and dispatch shared by tfft_c2c and tfft_c2c_noalloc.
// noalloc: the intermediate of a two-pass length goes to the device's
// scratch array, nothing is allocated (missing tables are reported, not
// built) and no launch is timed.
int c2c_impl(const void* x, void* y, long long N, long long batch, int dir, int precision,
             int ft_mode, double scale, tfft_ft_counts* counts, void* hip_stream, bool noalloc) {
    if (N < 1 || batch < 0) return TFFT_EINVAL;
    if (dir != TFFT_FORWARD && dir != TFFT_INVERSE) return TFFT_EINVAL;
    if (check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    if (ft_mode < TFFT_FT_OFF || ft_mode > TFFT_FT_THREAD) return TFFT_EINVAL;
    if (!(is_pow2(N) || (N % 3 == 0 && is_pow2(N / 3)))) return TFFT_EUNSUPPORTED;
    if (batch == 0) return TFFT_OK;
    if (!x || !y) return TFFT_EINVAL;
    if (ft_mode != TFFT_FT_OFF && !counts) return TFFT_EINVAL;
    const size_t S = precision == TFFT_FP32 ? 8 : 16;
    if (((uintptr_t)x % S) || ((uintptr_t)y % S)) return TFFT_EALIGN;
    // exact overlap (in place) is fine; partial overlap is not
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    const size_t bytes = (size_t)N * (size_t)batch * S;
    if (xb != yb && xb < yb + bytes && yb < xb + bytes) return TFFT_EINVAL;
    // one signal of a two-pass length must fit the scratch array
    if (noalloc && (size_t)N > TFFT_NOALLOC_SCRATCH_BYTES / S) return TFFT_ESCRATCH;
    if (scale == 0.0) scale = dir == TFFT_INVERSE ? 1.0 / (double)N : 1.0;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);

    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    // thread-level checking runs the kernels of ABFT mode 4 on the
    // correcting mode's route (single-pass lengths only)
    const bool thread_level = ft_mode == TFFT_FT_THREAD;
    const Tuning tu = get_tuning(precision, N, thread_level ? TFFT_FT_CORRECT : ft_mode);
    Route rt;
    if (!route_for(precision, N, thread_level ? 4 : ft_mode, &rt, tu.route)) return TFFT_EUNSUPPORTED;
    if (rt.single && ft_mode == TFFT_FT_CORRECT && x == y) {
        // in place: the kernel variant that keeps the right-side input sum
        rt.single = find_entry(precision, kSingle, N, 3, rt.single->variant);
        if (!rt.single) return TFFT_EUNSUPPORTED;
    }
    Inject inj = g_inj;
    if (inj.armed && (inj.precision != precision || inj.signal >= batch || inj.signal2 >= batch || inj.element >= N ||
                      !inject_fits(inj, rt.pass(0), rt.pass(1), rt.pass(2))))
        return TFFT_EINVAL;
    WsSource wsrc;
    if (noalloc) {
        int rc = scratch_for_device(current_device(), &wsrc.fixed);
        if (rc != TFFT_OK) return rc;
        wsrc.cap = TFFT_NOALLOC_SCRATCH_BYTES;
    }
    const bool may_alloc = !noalloc && !capturing(stream);
    int rc;
    if (precision == TFFT_FP32)
        rc = transform<float2>(rt, x, y, N, batch, dir, scale, counts, tu, inj, stream, may_alloc, wsrc);
    else
        rc = transform<double2>(rt, x, y, N, batch, dir, scale, counts, tu, inj, stream, may_alloc, wsrc);
    if (rc == TFFT_ECAPTURE && wsrc.fixed) rc = TFFT_ENOTPREPARED;
    if (rc == TFFT_OK) g_inj = Inject{};   // one-shot
    return rc;
}

}  // namespace

extern "C" {

int tfft_c2c(const void* x, void* y, long long N, long long batch, int dir, int precision,
             int ft_mode, double scale, tfft_ft_counts* counts, void* hip_stream) {
    return c2c_impl(x, y, N, batch, dir, precision, ft_mode, scale, counts, hip_stream, false);
}

int tfft_c2c_noalloc(const void* x, void* y, long long N, long long batch, int dir, int precision,
                     int ft_mode, double scale, tfft_ft_counts* counts, void* hip_stream) {
    return c2c_impl(x, y, N, batch, dir, precision, ft_mode, scale, counts, hip_stream, true);
}

int tfft_c2c_stepwise(const void* x, void* y, long long N, long long batch, int dir, int level,
                      void* hip_stream) {
    if (N < 2 || batch < 0 || (dir != TFFT_FORWARD && dir != TFFT_INVERSE) || level < 0 || level > 3)
        return TFFT_EINVAL;
    if (!is_pow2(N)) return TFFT_EUNSUPPORTED;
    if (batch == 0) return TFFT_OK;
    if (!x || !y) return TFFT_EINVAL;
    if (((uintptr_t)x % 8) || ((uintptr_t)y % 8)) return TFFT_EALIGN;
    const size_t bytes = (size_t)N * (size_t)batch * 8;
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    if (xb < yb + bytes && yb < xb + bytes) return TFFT_EINVAL;   // out of place only
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const double scale = dir == TFFT_INVERSE ? 1.0 / (double)N : 1.0;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    const bool may_alloc = !capturing(stream);
    if (level == 0) {
        // one launch per radix-2 stage, ping-pong so the last lands in y
        int S = 0;
        while ((1ll << S) < N) ++S;
        PassTwiddle* pt = nullptr;
        int rc = get_pass(TFFT_FP32, N, may_alloc, &pt);
        if (rc != TFFT_OK) return rc;
        void* ws = nullptr;
        if (S > 1) {
            rc = get_workspace(bytes, stream, may_alloc, &ws);
            if (rc != TFFT_OK) return rc;
        }
        const void* in = x;
        for (int st = 0; st < S; ++st) {
            void* out = ((S - 1 - st) % 2 == 0) ? y : ws;
            const hipError_t err =
                radix2_stage_launch(in, out, N, batch, 1ll << st, pt->hi, pt->lo, pt->bits,
                                    dir == TFFT_INVERSE ? 1 : 0, st == S - 1 ? (float)scale : 1.0f, stream);
            if (err != hipSuccess) return hip_fail(err);
            in = out;
        }
        return TFFT_OK;
    }
    if (level == 1) {
        static std::vector<KernelEntry>* r2 = nullptr;
        if (!r2) {
            r2 = new std::vector<KernelEntry>();
            register_fp32_stepwise(*r2);
        }
        const KernelEntry* e = nullptr;
        for (const KernelEntry& k : *r2)
            if (k.Ns == N) e = &k;
        if (!e) return TFFT_EUNSUPPORTED;
        SubTables* st = nullptr;
        int rc = get_sub(*e, may_alloc, &st);
        if (rc != TFFT_OK) return rc;
        Tuning tu = default_tuning(TFFT_FP32, N);
        tu.T = 1;
        tu.gran = 0;
        KArgs<float2> a{};
        fill_common(a, *e, *st, tu, nullptr);
        a.batch = batch;
        a.N = N;
        a.conj_in = a.conj_out = dir == TFFT_INVERSE ? 1 : 0;
        a.scale = (float)scale;
        a.x_intact = 1;
        return run<float2>(*e, x, y, a, (batch + e->slots_per_block - 1) / e->slots_per_block, stream);
    }
    // the library's plans without ABFT: level 2 the default route with the
    // default tuning, level 3 the tuned route
    const Tuning tu = level == 2 ? default_tuning(TFFT_FP32, N) : get_tuning(TFFT_FP32, N, TFFT_FT_OFF);
    Route rt;
    if (!route_for(TFFT_FP32, N, TFFT_FT_OFF, &rt, level == 2 ? 0 : tu.route)) return TFFT_EUNSUPPORTED;
    return transform<float2>(rt, x, y, N, batch, dir, scale, nullptr, tu, Inject{}, stream, may_alloc);
}

int tfft_c2c_offline(const void* x, void* y, long long N, long long batch, int dir, int precision,
                     double scale, tfft_ft_counts* counts, void* hip_stream) {
    if (N < 1 || batch < 0 || (dir != TFFT_FORWARD && dir != TFFT_INVERSE)) return TFFT_EINVAL;
    if (check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    if (!(is_pow2(N) || (N % 3 == 0 && is_pow2(N / 3)))) return TFFT_EUNSUPPORTED;
    if (batch == 0) return TFFT_OK;
    if (!x || !y || !counts) return TFFT_EINVAL;
    const size_t S = precision == TFFT_FP32 ? 8 : 16;
    if (((uintptr_t)x % S) || ((uintptr_t)y % S)) return TFFT_EALIGN;
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    const size_t bytes = (size_t)N * (size_t)batch * S;
    if (xb != yb && xb < yb + bytes && yb < xb + bytes) return TFFT_EINVAL;
    if (scale == 0.0) scale = dir == TFFT_INVERSE ? 1.0 / (double)N : 1.0;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);

    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    // the plain transform on the route tuned for it
    const Tuning tu = get_tuning(precision, N, TFFT_FT_OFF);
    Route rt;
    if (!route_for(precision, N, TFFT_FT_OFF, &rt, tu.route)) return TFFT_EUNSUPPORTED;
    if (g_inj.armed && (g_inj.precision != precision || g_inj.signal >= batch || g_inj.signal2 >= batch ||
                        g_inj.element >= N ||
                        !inject_fits(g_inj, rt.pass(0), rt.pass(1), rt.pass(2))))
        return TFFT_EINVAL;
    const bool may_alloc = !capturing(stream);
    const int dev = current_device();
    // full-length left vector
    void* left = nullptr;
    {
        auto key = std::make_tuple(precision, N, dev);
        auto it = g_left_full.find(key);
        if (it != g_left_full.end()) {
            left = it->second;
        } else {
            if (!may_alloc) return TFFT_ECAPTURE;
            int rc = precision == TFFT_FP32 ? build_left<float>(N, &left) : build_left<double>(N, &left);
            if (rc != TFFT_OK) return rc;
            g_left_full[key] = left;
        }
    }
    // workspace: p and q, energies, flags, right-side sums
    const long long groups = (batch + kOfflineT - 1) / kOfflineT;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    // p and q as complex double, energies as double (offline totals)
    const size_t off_nu = up(2 * (size_t)batch * 16), off_fl = off_nu + up((size_t)batch * 8);
    const size_t off_xs = off_fl + up((size_t)batch * 4);
    const size_t ws_bytes = off_xs + (size_t)groups * (size_t)N * S;
    void* ws = nullptr;
    switch (g_ws_off.get(dev, stream, ws_bytes, may_alloc, &ws)) {
        case WsResult::kOk: break;
        case WsResult::kWouldAllocate: return TFFT_ECAPTURE;
        default: return TFFT_ENOMEM;
    }
    char* w = static_cast<char*>(ws);
    OfflineArgs o{};
    o.x = x;
    o.y = y;
    o.N = N;
    o.batch = batch;
    o.left = left;
    o.M = N % 3 == 0 ? 5 : 3;
    o.conj = dir == TFFT_INVERSE ? 1 : 0;
    o.scale = scale;
    const double u = precision == TFFT_FP32 ? 0x1p-24 : 0x1p-53;
    const double kappa = get_tuning(precision, N, TFFT_FT_CORRECT).kappa;
    o.tau_coef = kappa * u * std::sqrt((double)N * std::log2((double)N));
    o.cs = w;
    o.nu = w + off_nu;
    o.flags = w + off_fl;
    o.xs = w + off_xs;
    o.counts = counts;
    const bool f32 = precision == TFFT_FP32;
    hipError_t e = f32 ? offline_launch<float2>(o, stream, 0) : offline_launch<double2>(o, stream, 0);
    if (e != hipSuccess) return hip_fail(e);
    // the plain transform (the hook, when armed, hits it), then W x_s
    const Inject inj = g_inj;
    int rc = f32 ? transform<float2>(rt, x, y, N, batch, dir, scale, nullptr, tu, inj, stream, may_alloc)
                 : transform<double2>(rt, x, y, N, batch, dir, scale, nullptr, tu, inj, stream, may_alloc);
    if (rc != TFFT_OK) return rc;
    const Inject none{};
    rc = f32 ? transform<float2>(rt, o.xs, o.xs, N, groups, TFFT_FORWARD, 1.0, nullptr, tu, none, stream, may_alloc)
             : transform<double2>(rt, o.xs, o.xs, N, groups, TFFT_FORWARD, 1.0, nullptr, tu, none, stream, may_alloc);
    if (rc != TFFT_OK) return rc;
    for (int step = 1; step <= 2; ++step) {
        e = f32 ? offline_launch<float2>(o, stream, step) : offline_launch<double2>(o, stream, step);
        if (e != hipSuccess) return hip_fail(e);
    }
    g_inj = Inject{};   // one-shot
    return TFFT_OK;
}

int tfft_ragged_supported(long long N, int precision) {
    if (precision != TFFT_FP32 || N < 1) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    RRoute r;
    return ragged_route(N, &r) ? 1 : 0;
}

int tfft_ragged_plan_create(tfft_ragged_plan* plan, const long long* sizes_host, long long count,
                            int precision) {
    if (!plan || count < 0 || (count > 0 && !sizes_host)) return TFFT_EINVAL;
    *plan = nullptr;
    if (check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    if (precision != TFFT_FP32) return TFFT_EUNSUPPORTED;
    for (long long i = 0; i < count; ++i)
        if (sizes_host[i] < 1) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    tfft_ragged_plan_s* P = new tfft_ragged_plan_s();
    P->device = current_device();
    P->precision = precision;
    P->waves = g_ragged_waves;
    int rc = ragged_build(P, sizes_host, count);
    if (rc != TFFT_OK) {
        if (P->buf) (void)hipFree(P->buf);
        if (P->ws) (void)hipFree(P->ws);
        delete P;
        return rc;
    }
    *plan = P;
    return TFFT_OK;
}

int tfft_ragged_plan_destroy(tfft_ragged_plan plan) {
    if (!plan) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (plan->buf) (void)hipFree(plan->buf);
    if (plan->ws) (void)hipFree(plan->ws);
    delete plan;
    return TFFT_OK;
}

int tfft_ragged_plan_info(tfft_ragged_plan plan, long long* info, int n) {
    if (!plan || !info || n < 1) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    long long v[10] = {plan->count, plan->total, plan->n_items, (long long)plan->classes.size(),
                       plan->ws_elems, 0, plan->n_batches, plan->window, 0, 0};
    RaggedKernel k = ragged_kernel(TFFT_FT_CORRECT, plan->waves);
    long long grid = (long long)k.blocks_per_cu * plan->cus;
    v[5] = grid < plan->n_items ? grid : plan->n_items;
    if (n > 8) {
        RQueue q{};
        hipError_t err = hipMemcpy(&q, plan->d_queue, sizeof(q), hipMemcpyDeviceToHost);
        if (err != hipSuccess) return hip_fail(err);
        v[8] = (long long)q.err_launches;
        v[9] = (long long)q.next;
    }
    for (int i = 0; i < n && i < 10; ++i) info[i] = v[i];
    return TFFT_OK;
}

int tfft_ragged_set_schedule(long long window_elems, long long item_elems, int waves) {
    if (window_elems < 0 || item_elems < 0 || (waves != 0 && waves != 3)) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_ragged_window = window_elems;
    if (item_elems > 0) g_ragged_item = item_elems;
    g_ragged_waves = waves;
    return TFFT_OK;
}

int tfft_ragged_test_wait(unsigned max_polls, unsigned extra) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_ragged_max_polls = max_polls;
    g_ragged_wait_extra = extra;
    return TFFT_OK;
}

int tfft_c2c_ragged(tfft_ragged_plan plan, const void* x, void* y, int dir, int unit_scale,
                    int mode, int ft_mode, tfft_ft_counts* counts, void* hip_stream) {
    if (!plan) return TFFT_EINVAL;
    if (dir != TFFT_FORWARD && dir != TFFT_INVERSE) return TFFT_EINVAL;
    if (mode != TFFT_RAGGED_PERSISTENT && mode != TFFT_RAGGED_PER_SIZE) return TFFT_EINVAL;
    if (ft_mode < TFFT_FT_OFF || ft_mode > TFFT_FT_CORRECT) return TFFT_EINVAL;
    if (plan->total == 0) return TFFT_OK;
    if (!x || !y) return TFFT_EINVAL;
    if (ft_mode != TFFT_FT_OFF && !counts) return TFFT_EINVAL;
    if (((uintptr_t)x % sizeof(float2)) || ((uintptr_t)y % sizeof(float2))) return TFFT_EALIGN;
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    const size_t bytes = (size_t)plan->total * sizeof(float2);
    if (xb != yb && xb < yb + bytes && yb < xb + bytes) return TFFT_EINVAL;
    // correction re-reads the inputs of single-pass and column-pass groups
    if (x == y && ft_mode == TFFT_FT_CORRECT) return TFFT_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    if (current_device() != plan->device) return TFFT_EINVAL;
    Inject inj = g_inj;
    if (inj.armed) {
        if (inj.precision != plan->precision || inj.signal >= plan->count ||
            inj.element >= plan->sizes[(size_t)inj.signal])
            return TFFT_EINVAL;
        // a second target must have the same length (same element numbering)
        if (inj.signal2 >= 0 && (inj.signal2 >= plan->count ||
                                 plan->sizes[(size_t)inj.signal2] != plan->sizes[(size_t)inj.signal]))
            return TFFT_EINVAL;
        RRoute rr;
        if (!ragged_route(plan->sizes[(size_t)inj.signal], &rr) ||
            !inject_fits(inj, rr.single ? rr.single : rr.col, rr.single ? nullptr : rr.row))
            return TFFT_EINVAL;
    }
    int rc = ragged_exec(plan, x, y, dir, unit_scale, mode, ft_mode, counts, inj, stream);
    if (rc == TFFT_OK) g_inj = Inject{};   // one-shot
    return rc;
}

}  // extern "C"
