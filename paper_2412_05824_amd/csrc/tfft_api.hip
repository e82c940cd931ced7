// tfft_api.hip -- host runtime behind the C ABI declared in include/tfft.h.
//
// Plans come from the compiled kernel registry; twiddle tables and the ABFT
// left vector e^T W are built here in long double, rounded once to the
// kernel precision, uploaded at prepare time and cached for the process.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tfft.h"
#include "tfft_registry.hpp"

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
    // angle = 2 pi m / den in [0, 2 pi); work with q = 8 m relative to den
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

struct Tables {
    void* tw = nullptr;     // device, concatenated stage tables
    void* left = nullptr;   // device, e^T W (N entries)
};

struct Tuning {
    int T;
    double kappa;
};

std::mutex g_mu;
std::vector<KernelEntry>* g_entries = nullptr;
std::map<std::tuple<int, long long, int>, const KernelEntry*> g_by_key;   // (prec, N, ft)
std::map<std::tuple<int, long long, int>, Tables> g_tables;              // (prec, N, device)
std::map<std::pair<int, long long>, Tuning> g_tuning;

struct Inject {
    bool armed = false;
    long long signal = -1, element = 0;
    int part = 0, bit = 0, precision = 0;
} g_inj;

bool g_stats = false;   // calibration mode: kernels record max |D0| / tau

void ensure_registry() {
    if (g_entries) return;
    g_entries = new std::vector<KernelEntry>();
    register_fp32(*g_entries);
    register_fp64(*g_entries);
    for (const KernelEntry& e : *g_entries) g_by_key[std::make_tuple(e.precision, (long long)e.N, e.ft)] = &e;
}

const KernelEntry* find_entry(int precision, long long N, int ft) {
    auto it = g_by_key.find(std::make_tuple(precision, N, ft));
    return it == g_by_key.end() ? nullptr : it->second;
}

Tuning default_tuning(int precision, long long N) {
    // fp32: small groups keep an undetected sub-threshold flip inside the
    // 2e-6 relative tolerance; fp64 has three orders of magnitude of margin.
    (void)N;
    if (precision == TFFT_FP32) return Tuning{4, 4.0};
    return Tuning{8, 16.0};
}

Tuning get_tuning(int precision, long long N) {
    auto it = g_tuning.find(std::make_pair(precision, N));
    return it == g_tuning.end() ? default_tuning(precision, N) : it->second;
}

template <class R> void put(std::vector<R>& v, long double re, long double im) {
    v.push_back((R)re);
    v.push_back((R)im);
}

template <class R> int build_tables(const KernelEntry& e, Tables* out) {
    const long long N = e.N;
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
        // w_M * w_N^n = exp(-2 pi i (N + M n) / (M N))
        long double wr, wi;
        cis_neg(N + M * n, M * N, &wr, &wi);
        const long double dr = 1.0L - wr, di = -wi;
        const long double den = dr * dr + di * di;
        put(left, (num_re * dr + num_im * di) / den, (num_im * dr - num_re * di) / den);
    }
    hipError_t err;
    err = hipMalloc(&out->tw, tw.size() * sizeof(R));
    if (err != hipSuccess) return (g_last_hip = (int)err, TFFT_ENOMEM);
    err = hipMalloc(&out->left, left.size() * sizeof(R));
    if (err != hipSuccess) return (g_last_hip = (int)err, TFFT_ENOMEM);
    err = hipMemcpy(out->tw, tw.data(), tw.size() * sizeof(R), hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err);
    err = hipMemcpy(out->left, left.data(), left.size() * sizeof(R), hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err);
    return TFFT_OK;
}

int current_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

// Tables for (precision, N) on the current device; builds them unless the
// stream is capturing.  Caller holds g_mu.
int get_tables(const KernelEntry& e, hipStream_t stream, bool allow_build, Tables** out) {
    auto key = std::make_tuple(e.precision, (long long)e.N, current_device());
    auto it = g_tables.find(key);
    if (it != g_tables.end()) { *out = &it->second; return TFFT_OK; }
    if (!allow_build) return TFFT_ECAPTURE;
    if (stream) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
            return TFFT_ECAPTURE;
    }
    Tables t;
    int rc = e.precision == TFFT_FP32 ? build_tables<float>(e, &t) : build_tables<double>(e, &t);
    if (rc != TFFT_OK) return rc;
    g_tables[key] = t;
    *out = &g_tables[key];
    return TFFT_OK;
}

template <class V>
int launch_transform(const KernelEntry& e, const Tables& tb, const void* x, void* y, long long batch,
                     int dir, double scale, tfft_ft_counts* counts, const Tuning& tu,
                     const Inject& inj, hipStream_t stream) {
    using R = typename RealOf<V>::type;
    KArgs<V> a{};
    a.tw = static_cast<const V*>(tb.tw);
    a.left = static_cast<const V*>(tb.left);
    a.batch = batch;
    a.T = tu.T;
    a.conj = dir == TFFT_INVERSE ? 1 : 0;
    a.scale = (R)scale;
    const double u = e.precision == TFFT_FP32 ? 0x1p-24 : 0x1p-53;
    const double N = (double)e.N;
    a.tau_coef = (R)(tu.kappa * u * std::sqrt(N * std::log2(N)));
    a.cap = e.precision == TFFT_FP32 ? (R)0x1p64 : (R)0x1p512;
    a.counts = reinterpret_cast<FtCounts*>(counts);
    a.inj_signal = inj.armed ? inj.signal : -1;
    a.inj_elem = (int)inj.element;
    a.inj_part = inj.part;
    a.inj_bit = inj.bit;
    a.stats = g_stats ? 1 : 0;
    a.x_intact = x != y ? 1 : 0;
    const long long per_block = (long long)e.slots_per_block * tu.T;
    const long long grid = (batch + per_block - 1) / per_block;
    if (grid > 0x7fffffffLL) return TFFT_EUNSUPPORTED;
    hipError_t err = e.launch(x, y, &a, grid, stream);
    if (err != hipSuccess) return hip_fail(err);
    return TFFT_OK;
}

bool is_pow2(long long n) { return n > 0 && (n & (n - 1)) == 0; }

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
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    return find_entry(precision, N, 0) != nullptr ? 1 : 0;
}

int tfft_prepare(long long N, int precision, int ft_mode) {
    if (N < 1 || (precision != TFFT_FP32 && precision != TFFT_FP64) || ft_mode < 0 || ft_mode > 2)
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_registry();
    const KernelEntry* e = find_entry(precision, N, ft_mode);
    if (!e) return TFFT_EUNSUPPORTED;
    Tables* tb = nullptr;
    return get_tables(*e, nullptr, true, &tb);
}

int tfft_set_tuning(long long N, int precision, int T, double kappa) {
    if (N < 1 || (precision != TFFT_FP32 && precision != TFFT_FP64) || T < 0 || T > 32 || kappa < 0)
        return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Tuning tu = get_tuning(precision, N);
    if (T > 0) tu.T = T;
    if (kappa > 0) tu.kappa = kappa;
    g_tuning[std::make_pair(precision, N)] = tu;
    return TFFT_OK;
}

int tfft_get_tuning(long long N, int precision, int* T, double* kappa) {
    if (!T || !kappa || (precision != TFFT_FP32 && precision != TFFT_FP64)) return TFFT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Tuning tu = get_tuning(precision, N);
    *T = tu.T;
    *kappa = tu.kappa;
    return TFFT_OK;
}

int tfft_inject_arm(long long signal, long long element, int part, int bit, int precision) {
    if (signal < 0 || element < 0 || (part != 0 && part != 1)) return TFFT_EINVAL;
    if (precision != TFFT_FP32 && precision != TFFT_FP64) return TFFT_EINVAL;
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

int tfft_calibration(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_stats = on != 0;
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
    if (precision != TFFT_FP32 && precision != TFFT_FP64) return TFFT_EINVAL;
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
    const KernelEntry* e = find_entry(precision, N, ft_mode);
    if (!e) return TFFT_EUNSUPPORTED;
    Inject inj = g_inj;
    if (inj.armed) {
        if (inj.precision != precision || inj.signal >= batch || inj.element >= N) return TFFT_EINVAL;
    }
    Tables* tb = nullptr;
    int rc = get_tables(*e, stream, true, &tb);
    if (rc != TFFT_OK) return rc;
    const Tuning tu = get_tuning(precision, N);
    if (precision == TFFT_FP32)
        rc = launch_transform<float2>(*e, *tb, x, y, batch, dir, scale, counts, tu, inj, stream);
    else
        rc = launch_transform<double2>(*e, *tb, x, y, batch, dir, scale, counts, tu, inj, stream);
    if (rc == TFFT_OK) g_inj = Inject{};   // one-shot
    return rc;
}

int tfft_c2c_ragged(const void*, void*, const long long*, const long long*, long long, int, int,
                    int, tfft_ft_counts*, void*) {
    return TFFT_EUNSUPPORTED;
}

int tfft_prepare_ragged(const long long*, long long, int, int) { return TFFT_EUNSUPPORTED; }

}  // extern "C"
