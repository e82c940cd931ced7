// Kernels of the stepwise study without ABFT (Sec. 5.1, the v0 -> v3 chain of
// the transform alone): level 0 launches one kernel per radix-2 stage that
// reads and writes global memory; level 1 runs every radix-2 stage in one
// kernel, exchanging through LDS.  Levels 2 and 3 are the library's own
// plans (default and tuned), run by the host entry point.
#include "tfft_registry.hpp"

namespace tfft {

// One radix-2 Stockham stage of sub-length L over a batch of N-point
// signals: butterfly (j, k), j < N / 2L, k < L, reads x[jL + k] and
// x[jL + k + N/2] and writes y[2jL + k] and y[2jL + k + L], the second input
// times w_{2L}^k = w_N^{k N / 2L} (two-level table; conjugated for the
// inverse).  The last stage scales.
__global__ __launch_bounds__(256) void k_radix2_stage(const float2* __restrict__ x, float2* __restrict__ y,
                                                      long long N, long long total, long long L,
                                                      const float2* __restrict__ hi,
                                                      const float2* __restrict__ lo, int bits, int conj,
                                                      float scale) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const long long half = N / 2;
    const long long b = i / half, r = i % half;
    const long long k = r % L, j = r / L;
    const float2* xb = x + b * N;
    float2* yb = y + b * N;
    const float2 u = xb[j * L + k];
    const float2 v = xb[j * L + k + half];
    const unsigned long long m = (unsigned long long)(k * (half / L));   // < N / 2
    const float2 h = hi[m >> bits], l = lo[m & ((1ull << bits) - 1ull)];
    float2 w = float2{h.x * l.x - h.y * l.y, h.x * l.y + h.y * l.x};
    if (conj) w.y = -w.y;
    const float2 t = float2{v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
    yb[j * 2 * L + k] = float2{(u.x + t.x) * scale, (u.y + t.y) * scale};
    yb[j * 2 * L + k + L] = float2{(u.x - t.x) * scale, (u.y - t.y) * scale};
}

hipError_t radix2_stage_launch(const void* x, void* y, long long N, long long batch, long long L,
                               const void* hi, const void* lo, int bits, int conj, float scale,
                               hipStream_t s) {
    const long long total = batch * (N / 2);
    const long long grid = (total + 255) / 256;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_radix2_stage, dim3((unsigned)grid), dim3(256), 0, s, static_cast<const float2*>(x),
                       static_cast<float2*>(y), N, total, L, static_cast<const float2*>(hi),
                       static_cast<const float2*>(lo), bits, conj, scale);
    return hipGetLastError();
}

// Level 1: one kernel, radix-2 stages through LDS (lanes of E / 2
// butterflies; E grows with the length so a signal fits one workgroup).
template <int Ns, int E, int WC, int... Rs> static void add_r2(std::vector<KernelEntry>& out) {
    using PL = Plan<kSingle, Ns, E, WC, 4, Rs...>;
    out.push_back(make_entry<float2, PL, 0, false, Rs...>(0));
}

void register_fp32_stepwise(std::vector<KernelEntry>& out) {
    add_r2<64, 2, 4, 2, 2, 2, 2, 2, 2>(out);
    add_r2<128, 2, 4, 2, 2, 2, 2, 2, 2, 2>(out);
    add_r2<256, 2, 4, 2, 2, 2, 2, 2, 2, 2, 2>(out);
    add_r2<512, 2, 4, 2, 2, 2, 2, 2, 2, 2, 2, 2>(out);
    add_r2<1024, 2, 4, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2>(out);
    add_r2<2048, 2, 4, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2>(out);
    add_r2<4096, 4, 4, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2>(out);
    add_r2<8192, 8, 4, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2>(out);
}

}  // namespace tfft
