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
#include <tuple>
#include <vector>

#include "tfft.h"
#include "tfft_ragged.hpp"

using namespace tfft;

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

struct SubTables { void* tw = nullptr; void* left = nullptr; };
struct PassTwiddle { void* hi = nullptr; void* lo = nullptr; int bits = 0; };
struct Workspace { void* ptr = nullptr; size_t bytes = 0; };

struct Tuning {
    int T;
    double kappa;
    long long chunk_bytes;
};

std::mutex g_mu;
std::vector<KernelEntry>* g_entries = nullptr;
std::map<std::tuple<int, int, int, int>, const KernelEntry*> g_by_key;   // (prec, kind, Ns, ft)
std::map<std::pair<int, int>, const KernelEntry*> g_ragged_by_key;      // (ragged plan id, ft)
std::map<std::tuple<int, int, int, long long>, SubTables> g_sub;         // (prec, Ns, device, radices)
std::map<std::tuple<int, long long, int>, PassTwiddle> g_pass;           // (prec, N, device)
std::map<int, Workspace> g_ws;                                           // device
std::map<std::pair<int, long long>, Tuning> g_tuning;

struct Inject {
    bool armed = false;
    long long signal = -1, element = 0;
    int part = 0, bit = 0, precision = 0;
} g_inj;

bool g_stats = false;   // calibration mode: kernels record max |D0| / tau

// Optional per-launch timing: a HIP event pair around every kernel launch, on
// the launch stream, with the launch's algorithmic bytes (input + output).
struct LaunchRec {
    const KernelEntry* e;
    hipEvent_t start, stop;
    double bytes;
};
bool g_prof = false;
std::vector<LaunchRec> g_prof_log;
std::string g_prof_text;   // aggregated, not yet read

void ensure_registry() {
    if (g_entries) return;
    g_entries = new std::vector<KernelEntry>();
    register_fp32_single(*g_entries);
    register_fp32_tiles(*g_entries);
    register_fp64_single(*g_entries);
    register_fp64_tiles(*g_entries);
    register_fp32_ragged_single(*g_entries);
    register_fp32_ragged_tiles(*g_entries);
    for (const KernelEntry& e : *g_entries) {
        if (e.ragged_id >= 0) g_ragged_by_key[std::make_pair(e.ragged_id, e.ft)] = &e;
        else g_by_key[std::make_tuple(e.precision, e.kind, e.Ns, e.ft)] = &e;
    }
}

const KernelEntry* find_entry(int precision, int kind, long long Ns, int ft) {
    if (Ns > (1 << 30)) return nullptr;
    auto it = g_by_key.find(std::make_tuple(precision, kind, (int)Ns, ft));
    return it == g_by_key.end() ? nullptr : it->second;
}

// How a length is executed: one single-pass kernel, or a column pass of
// length N1 and a row pass of length N2.
struct Route {
    const KernelEntry* single = nullptr;
    const KernelEntry* col = nullptr;
    const KernelEntry* row = nullptr;
    long long N1 = 0, N2 = 0;
};

bool route_for(int precision, long long N, int ft, Route* r) {
    *r = Route{};
    if ((r->single = find_entry(precision, kSingle, N, ft))) return true;
    // balanced split N = N1 * N2 with N1 <= N2, both with tile kernels
    long long best1 = 0;
    for (long long n1 = 2; n1 * n1 <= N; n1 <<= 1) {
        if (N % n1) continue;
        const long long n2 = N / n1;
        if (find_entry(precision, kColPass, n1, ft) && find_entry(precision, kRowPass, n2, ft)) best1 = n1;
    }
    if (!best1) return false;
    r->N1 = best1;
    r->N2 = N / best1;
    r->col = find_entry(precision, kColPass, r->N1, ft);
    r->row = find_entry(precision, kRowPass, r->N2, ft);
    return true;
}

Tuning default_tuning(int precision, long long N) {
    // Groups of T signals share one checksum reduction (Sec. 4.3).  In fp32 an
    // undetected flip just under the threshold perturbs one signal by about
    // kappa * u * sqrt(T log2 Ns) of its norm, so T stays small to keep that
    // under the 2e-6 relative tolerance; fp64 has ample margin.
    Tuning t{};
    t.chunk_bytes = 128ll << 20;
    if (precision == TFFT_FP32) {
        t.kappa = 8.0;
        t.T = N <= 128 ? 2 : 1;
    } else {
        t.kappa = 16.0;
        t.T = 8;
    }
    return t;
}

Tuning get_tuning(int precision, long long N) {
    auto it = g_tuning.find(std::make_pair(precision, N));
    return it == g_tuning.end() ? default_tuning(precision, N) : it->second;
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
    // a_n = (1 - w_M^N) / (1 - w_M w_N^n), w_M = exp(-2 pi i / M)
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
    int rc = upload(tw, &out->tw);
    if (rc != TFFT_OK) return rc;
    return upload(left, &out->left);
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
    long long sig = 0;
    for (int s = 0; s < e.n_stages; ++s) sig = sig * 32 + e.radices[s];
    return sig;
}

int get_sub(const KernelEntry& e, bool may_alloc, SubTables** out) {
    auto key = std::make_tuple(e.precision, e.Ns, current_device(), radix_signature(e));
    auto it = g_sub.find(key);
    if (it != g_sub.end()) { *out = &it->second; return TFFT_OK; }
    if (!may_alloc) return TFFT_ECAPTURE;
    SubTables t;
    int rc = e.precision == TFFT_FP32 ? build_sub<float>(e, &t) : build_sub<double>(e, &t);
    if (rc != TFFT_OK) return rc;
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

int get_workspace(size_t bytes, bool may_alloc, void** out) {
    Workspace& w = g_ws[current_device()];
    if (w.bytes >= bytes) { *out = w.ptr; return TFFT_OK; }
    if (!may_alloc) return TFFT_ECAPTURE;
    if (w.ptr) {
        hipError_t e = hipDeviceSynchronize();   // no kernel may still use the old buffer
        if (e != hipSuccess) return hip_fail(e);
        (void)hipFree(w.ptr);
        w = Workspace{};
    }
    hipError_t e = hipMalloc(&w.ptr, bytes);
    if (e != hipSuccess) { g_last_hip = (int)e; w = Workspace{}; return TFFT_ENOMEM; }
    w.bytes = bytes;
    *out = w.ptr;
    return TFFT_OK;
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
    a.T = tu.T;
    const double u = e.precision == TFFT_FP32 ? 0x1p-24 : 0x1p-53;
    const double Ns = (double)e.Ns;
    a.tau_coef = (R)(tu.kappa * u * std::sqrt(Ns * std::log2(Ns)));
    a.cap = e.precision == TFFT_FP32 ? (R)0x1p64 : (R)0x1p512;
    a.counts = reinterpret_cast<FtCounts*>(counts);
    a.inj_signal = -1;
    a.stats = g_stats ? 1 : 0;
}

template <class V> int run(const KernelEntry& e, const void* x, void* y, const KArgs<V>& a,
                           long long grid, hipStream_t stream) {
    if (grid <= 0) return TFFT_OK;
    if (grid > 0x7fffffffLL) return TFFT_EUNSUPPORTED;
    LaunchRec rec{};
    const bool prof = g_prof && !capturing(stream);
    if (prof) {
        rec.e = &e;
        rec.bytes = 2.0 * (double)a.batch * (double)a.N * (double)sizeof(V);
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

template <class V>
int transform(const Route& rt, const void* x, void* y, long long N, long long batch, int dir,
              double scale, tfft_ft_counts* counts, const Tuning& tu, const Inject& inj,
              hipStream_t stream, bool may_alloc) {
    using R = typename RealOf<V>::type;
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
        if (inj.armed) { a.inj_signal = inj.signal; a.inj_elem = inj.element; a.inj_part = inj.part; a.inj_bit = inj.bit; }
        const long long per_block = (long long)rt.single->slots_per_block * tu.T;
        return run<V>(*rt.single, x, y, a, (batch + per_block - 1) / per_block, stream);
    }
    // two passes over chunks of signals
    SubTables *sa = nullptr, *sb = nullptr;
    PassTwiddle* pt = nullptr;
    int rc = get_sub(*rt.col, may_alloc, &sa);
    if (rc == TFFT_OK) rc = get_sub(*rt.row, may_alloc, &sb);
    if (rc == TFFT_OK) rc = get_pass(precision, N, may_alloc, &pt);
    if (rc != TFFT_OK) return rc;
    const size_t sig_bytes = (size_t)N * sizeof(V);
    long long chunk = tu.chunk_bytes / (long long)sig_bytes;
    if (chunk < 1) chunk = 1;
    if (chunk > batch) chunk = batch;
    void* ws = nullptr;
    rc = get_workspace((size_t)chunk * sig_bytes, may_alloc, &ws);
    if (rc != TFFT_OK) return rc;

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
        B.inj_signal = -1;
        if (inj.armed && inj.signal >= c0 && inj.signal < c0 + cnt) {
            B.inj_signal = inj.signal;   // global index: the kernel compares sig_base + s
            B.inj_elem = inj.element;
            B.inj_part = inj.part;
            B.inj_bit = inj.bit;
        }
        const long long groups = (cnt + tu.T - 1) / tu.T;
        rc = run<V>(*rt.col, xb + (size_t)c0 * sig_bytes, ws, A, groups * A.tiles, stream);
        if (rc != TFFT_OK) return rc;
        rc = run<V>(*rt.row, ws, yb + (size_t)c0 * sig_bytes, B, groups * B.tiles, stream);
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

RaggedKernel ragged_kernel(int ft) {
    static RaggedKernel k[3];
    static bool done[3] = {false, false, false};
    if (!done[ft]) {
        k[ft] = ft == 0 ? ragged_kernel_ft0() : ft == 1 ? ragged_kernel_ft1() : ragged_kernel_ft2();
        done[ft] = true;
    }
    return k[ft];
}

}  // namespace

struct tfft_ragged_plan_s {
    int device = 0;
    int precision = TFFT_FP32;
    long long count = 0, total = 0, ws_elems = 0;
    std::vector<long long> sizes;          // host copy, for argument checks
    std::vector<RClass> classes;           // host copy (per-size launches)
    std::vector<int> order;                // launch order of the classes (per-size mode)
    long long n_items = 0;
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

    // classes: one per length (single) or two (column pass, row pass)
    std::map<long long, std::vector<long long>, std::greater<long long>> by_len;
    for (long long i = 0; i < count; ++i) by_len[sizes[i]].push_back(i);
    struct Pending { RRoute rt; std::vector<long long> ids; };
    std::vector<Pending> lens;
    for (auto& kv : by_len) {
        Pending pd;
        if (!ragged_route(kv.first, &pd.rt)) return TFFT_EUNSUPPORTED;
        pd.ids = kv.second;
        lens.push_back(std::move(pd));
    }
    // host tables: ids, x offsets, workspace offsets, per length
    std::vector<long long> tab;
    long long ws_tot = 0, groups_tot = 0;
    struct Made { RClass cl; size_t ids_at, xoff_at, wsoff_at; bool two; };
    std::vector<Made> made;   // single classes and column passes first, row passes after
    std::vector<Made> rows;
    for (Pending& pd : lens) {
        const long long N = pd.rt.single ? pd.rt.single->Ns : pd.rt.N1 * pd.rt.N2;
        const long long n = (long long)pd.ids.size();
        const Tuning tu = get_tuning(TFFT_FP32, N);
        const size_t ids_at = tab.size();
        for (long long i : pd.ids) tab.push_back(i);
        const size_t xoff_at = tab.size();
        for (long long i : pd.ids) tab.push_back(xoff[i]);
        const long long groups = (n + tu.T - 1) / tu.T;
        if (pd.rt.single) {
            const KernelEntry& e = *pd.rt.single;
            SubTables* st = nullptr;
            int rc = get_sub(e, true, &st);
            if (rc != TFFT_OK) return rc;
            RClass c{};
            fill_common(c.args, e, *st, tu, nullptr);
            c.args.batch = n;
            c.args.N = N;
            c.args.x_intact = 1;
            c.plan = e.ragged_id;
            c.final_pass = 1;
            const long long per_block = (long long)e.slots_per_block * tu.T;
            c.nblocks = (int)((n + per_block - 1) / per_block);
            c.cnt_base = -1;
            made.push_back(Made{c, ids_at, xoff_at, xoff_at, false});
            continue;
        }
        const size_t wsoff_at = tab.size();
        for (long long j = 0; j < n; ++j) { tab.push_back(ws_tot); ws_tot += N; }
        SubTables *sa = nullptr, *sb = nullptr;
        PassTwiddle* pt = nullptr;
        int rc = get_sub(*pd.rt.col, true, &sa);
        if (rc == TFFT_OK) rc = get_sub(*pd.rt.row, true, &sb);
        if (rc == TFFT_OK) rc = get_pass(TFFT_FP32, N, true, &pt);
        if (rc != TFFT_OK) return rc;
        RClass A{}, B{};
        fill_common(A.args, *pd.rt.col, *sa, tu, nullptr);
        fill_common(B.args, *pd.rt.row, *sb, tu, nullptr);
        for (RClass* k : {&A, &B}) {
            k->args.batch = n;
            k->args.N = N;
            k->args.N1 = (int)pd.rt.N1;
            k->args.N2 = (int)pd.rt.N2;
            k->args.x_intact = 1;
            k->cnt_base = (int)groups_tot;
        }
        B.args.tw_hi = static_cast<const float2*>(pt->hi);
        B.args.tw_lo = static_cast<const float2*>(pt->lo);
        B.args.tw_bits = pt->bits;
        A.args.tiles = A.tiles = (int)(pd.rt.N2 / pd.rt.col->slots_per_block);
        B.args.tiles = B.tiles = (int)(pd.rt.N1 / pd.rt.row->slots_per_block);
        A.plan = pd.rt.col->ragged_id;
        B.plan = pd.rt.row->ragged_id;
        A.dst_ws = 1;
        A.signal_after = 1;
        B.src_ws = 1;
        B.final_pass = 1;
        B.need = A.tiles;
        A.nblocks = (int)(groups * A.tiles);
        B.nblocks = (int)(groups * B.tiles);
        if ((long long)A.nblocks != groups * A.tiles || (long long)B.nblocks != groups * B.tiles)
            return TFFT_EUNSUPPORTED;
        groups_tot += groups;
        // column passes go first in the queue
        made.insert(made.begin(), Made{A, ids_at, xoff_at, wsoff_at, true});
        rows.push_back(Made{B, ids_at, wsoff_at, xoff_at, true});
    }
    for (Made& m : rows) made.push_back(m);
    // the column passes were inserted at the front in reverse: largest first
    {
        size_t ncol = 0;
        while (ncol < made.size() && made[ncol].cl.signal_after) ++ncol;
        std::reverse(made.begin(), made.begin() + ncol);
    }
    P->ws_elems = ws_tot;

    // items, in class order
    std::vector<RItem> items;
    for (size_t c = 0; c < made.size(); ++c)
        for (int b = 0; b < made[c].cl.nblocks; ++b) items.push_back(RItem{(int)c, b});
    P->n_items = (long long)items.size();

    // one device buffer: classes | items | desc | queue | cnt_a | cnt_b | tables
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t o_cls = 0;
    const size_t o_items = al(o_cls + made.size() * sizeof(RClass));
    const size_t o_desc = al(o_items + items.size() * sizeof(RItem));
    const size_t o_q = al(o_desc + sizeof(RaggedDesc));
    const size_t o_ca = al(o_q + sizeof(RQueue));
    const size_t o_cb = al(o_ca + (size_t)groups_tot * sizeof(unsigned));
    const size_t o_tab = al(o_cb + (size_t)groups_tot * sizeof(unsigned));
    const size_t bytes = al(o_tab + tab.size() * sizeof(long long));
    hipError_t err = hipMalloc(&P->buf, bytes);
    if (err != hipSuccess) { g_last_hip = (int)err; P->buf = nullptr; return TFFT_ENOMEM; }
    if (ws_tot > 0) {
        err = hipMalloc(&P->ws, (size_t)ws_tot * sizeof(float2));
        if (err != hipSuccess) { g_last_hip = (int)err; P->ws = nullptr; return TFFT_ENOMEM; }
    }
    char* base = static_cast<char*>(P->buf);
    const long long* dtab = reinterpret_cast<const long long*>(base + o_tab);
    for (Made& m : made) {
        m.cl.args.id_tab = dtab + m.ids_at;
        m.cl.args.in_tab = dtab + m.xoff_at;
        m.cl.args.out_tab = dtab + m.wsoff_at;
    }
    P->classes.clear();
    for (Made& m : made) P->classes.push_back(m.cl);
    RaggedDesc desc{};
    desc.classes = reinterpret_cast<const RClass*>(base + o_cls);
    desc.items = reinterpret_cast<const RItem*>(base + o_items);
    desc.n_items = P->n_items;
    desc.q = reinterpret_cast<RQueue*>(base + o_q);
    desc.cnt_a = reinterpret_cast<unsigned*>(base + o_ca);
    desc.cnt_b = reinterpret_cast<unsigned*>(base + o_cb);
    desc.ws = static_cast<float2*>(P->ws);
    P->d_desc = reinterpret_cast<RaggedDesc*>(base + o_desc);
    P->d_queue = desc.q;

    std::vector<char> host(bytes, 0);
    memcpy(host.data() + o_cls, P->classes.data(), P->classes.size() * sizeof(RClass));
    memcpy(host.data() + o_items, items.data(), items.size() * sizeof(RItem));
    memcpy(host.data() + o_desc, &desc, sizeof(desc));
    memcpy(host.data() + o_tab, tab.data(), tab.size() * sizeof(long long));
    err = hipMemcpy(P->buf, host.data(), bytes, hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err);

    hipDeviceProp_t prop{};
    err = hipGetDeviceProperties(&prop, P->device);
    if (err != hipSuccess) return hip_fail(err);
    P->cus = prop.multiProcessorCount;
    return TFFT_OK;
}

int ragged_exec(tfft_ragged_plan_s* P, const void* x, void* y, int dir, int unit_scale, int mode,
                int ft, tfft_ft_counts* counts, const Inject& inj, hipStream_t stream) {
    RaggedCall c{};
    c.x = static_cast<const float2*>(x);
    c.y = static_cast<float2*>(y);
    c.counts = reinterpret_cast<FtCounts*>(counts);
    c.inj_signal = inj.armed ? inj.signal : -1;
    c.inj_elem = inj.element;
    c.inj_part = inj.part;
    c.inj_bit = inj.bit;
    c.conj = dir == TFFT_INVERSE ? 1 : 0;
    c.unit_scale = unit_scale ? 1 : 0;
    c.stats = g_stats ? 1 : 0;
    if (P->n_items == 0) return TFFT_OK;
    if (mode == TFFT_RAGGED_PERSISTENT) {
        const RaggedKernel k = ragged_kernel(ft);
        if (!k.launch || k.blocks_per_cu <= 0) return TFFT_EUNSUPPORTED;
        long long grid = (long long)k.blocks_per_cu * P->cus;
        if (grid > P->n_items) grid = P->n_items;
        LaunchRec rec{};
        const bool prof = g_prof && !capturing(stream);
        if (prof) {
            KernelEntry& pe = g_ragged_prof_entry[ft];
            pe.precision = TFFT_FP32;
            pe.kind = 3;
            pe.Ns = 0;
            pe.ft = ft;
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
        a.inj_signal = cl.final_pass ? c.inj_signal : -1;
        a.inj_elem = c.inj_elem;
        a.inj_part = c.inj_part;
        a.inj_bit = c.inj_bit;
        const void* src = cl.src_ws ? P->ws : x;
        void* dst = cl.dst_ws ? P->ws : y;
        int rc = run<float2>(*e, src, dst, a, cl.nblocks, stream);
        if (rc != TFFT_OK) return rc;
    }
    return TFFT_OK;
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

int tfft_prepare(long long N, int precision, int ft_mode) {
    if (N < 1 || check_precision(precision) != TFFT_OK || ft_mode < 0 || ft_mode > 2) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    Route r;
    if (!route_for(precision, N, ft_mode, &r)) return TFFT_EUNSUPPORTED;
    SubTables* st = nullptr;
    if (r.single) return get_sub(*r.single, true, &st);
    int rc = get_sub(*r.col, true, &st);
    if (rc == TFFT_OK) rc = get_sub(*r.row, true, &st);
    PassTwiddle* pt = nullptr;
    if (rc == TFFT_OK) rc = get_pass(precision, N, true, &pt);
    return rc;
}

int tfft_set_tuning(long long N, int precision, int T, double kappa) {
    if (N < 1 || check_precision(precision) != TFFT_OK || T < 0 || T > 32 || kappa < 0) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Tuning tu = get_tuning(precision, N);
    if (T > 0) tu.T = T;
    if (kappa > 0) tu.kappa = kappa;
    g_tuning[std::make_pair(precision, N)] = tu;
    return TFFT_OK;
}

int tfft_get_tuning(long long N, int precision, int* T, double* kappa) {
    if (!T || !kappa || check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Tuning tu = get_tuning(precision, N);
    *T = tu.T;
    *kappa = tu.kappa;
    return TFFT_OK;
}

int tfft_set_chunk(long long N, int precision, long long chunk_bytes) {
    if (N < 1 || check_precision(precision) != TFFT_OK || chunk_bytes < 0) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Tuning tu = get_tuning(precision, N);
    if (chunk_bytes > 0) tu.chunk_bytes = chunk_bytes;
    g_tuning[std::make_pair(precision, N)] = tu;
    return TFFT_OK;
}

int tfft_profile(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof = on != 0;
    return TFFT_OK;
}

int tfft_profile_read(char* buf, long long buflen) {
    std::lock_guard<std::mutex> lk(g_mu);
    // aggregate the pending launches per kernel: launches, total ms, bytes
    struct Agg { long long n = 0; double ms = 0, bytes = 0; };
    std::map<std::tuple<int, int, int, int>, Agg> agg;
    for (LaunchRec& r : g_prof_log) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            Agg& g = agg[std::make_tuple(r.e->precision, r.e->kind, r.e->Ns, r.e->ft)];
            g.n += 1;
            g.ms += ms;
            g.bytes += r.bytes;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof_log.clear();
    static const char* kinds[] = {"single", "colpass", "rowpass", "ragged"};
    for (auto& kv : agg) {
        char line[256];
        snprintf(line, sizeof(line), "%s %s %d %d %lld %.6f %.1f\n",
                 std::get<0>(kv.first) == TFFT_FP32 ? "fp32" : "fp64", kinds[std::get<1>(kv.first)],
                 std::get<2>(kv.first), std::get<3>(kv.first), kv.second.n, kv.second.ms, kv.second.bytes);
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

int tfft_inject_arm(long long signal, long long element, int part, int bit, int precision) {
    if (signal < 0 || element < 0 || (part != 0 && part != 1)) return TFFT_EINVAL;
    if (check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    const int width = precision == TFFT_FP32 ? 32 : 64;
    if (bit < 0 || bit >= width) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_inj.armed = true;
    g_inj.signal = signal;
    g_inj.element = element;
    g_inj.part = part;
    g_inj.bit = bit;
    g_inj.precision = precision;
    return TFFT_OK;
}

int tfft_inject_disarm(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_inj = Inject{};
    return TFFT_OK;
}

int tfft_c2c(const void* x, void* y, long long N, long long batch, int dir, int precision,
             int ft_mode, double scale, tfft_ft_counts* counts, void* hip_stream) {
    if (N < 1 || batch < 0) return TFFT_EINVAL;
    if (dir != TFFT_FORWARD && dir != TFFT_INVERSE) return TFFT_EINVAL;
    if (check_precision(precision) != TFFT_OK) return TFFT_EINVAL;
    if (ft_mode < TFFT_FT_OFF || ft_mode > TFFT_FT_CORRECT) return TFFT_EINVAL;
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
    if (scale == 0.0) scale = dir == TFFT_INVERSE ? 1.0 / (double)N : 1.0;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);

    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    Route rt;
    if (!route_for(precision, N, ft_mode, &rt)) return TFFT_EUNSUPPORTED;
    if (rt.single && ft_mode == TFFT_FT_CORRECT && x == y) {
        // in place: the kernel variant that keeps the right-side input sum
        rt.single = find_entry(precision, kSingle, N, 3);
        if (!rt.single) return TFFT_EUNSUPPORTED;
    }
    Inject inj = g_inj;
    if (inj.armed && (inj.precision != precision || inj.signal >= batch || inj.element >= N))
        return TFFT_EINVAL;
    const bool may_alloc = !capturing(stream);
    const Tuning tu = get_tuning(precision, N);
    int rc;
    if (precision == TFFT_FP32)
        rc = transform<float2>(rt, x, y, N, batch, dir, scale, counts, tu, inj, stream, may_alloc);
    else
        rc = transform<double2>(rt, x, y, N, batch, dir, scale, counts, tu, inj, stream, may_alloc);
    if (rc == TFFT_OK) g_inj = Inject{};   // one-shot
    return rc;
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
    long long v[8] = {plan->count, plan->total, plan->n_items, (long long)plan->classes.size(),
                      plan->ws_elems, 0, 0, 0};
    RaggedKernel k = ragged_kernel(TFFT_FT_CORRECT);
    long long grid = (long long)k.blocks_per_cu * plan->cus;
    v[5] = grid < plan->n_items ? grid : plan->n_items;
    if (n > 6) {
        RQueue q{};
        hipError_t err = hipMemcpy(&q, plan->d_queue, sizeof(q), hipMemcpyDeviceToHost);
        if (err != hipSuccess) return hip_fail(err);
        v[6] = (long long)q.err;
        v[7] = (long long)q.next;
    }
    for (int i = 0; i < n && i < 8; ++i) info[i] = v[i];
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
    }
    int rc = ragged_exec(plan, x, y, dir, unit_scale, mode, ft_mode, counts, inj, stream);
    if (rc == TFFT_OK) g_inj = Inject{};   // one-shot
    return rc;
}

}  // extern "C"
