// tfft_offline.hip -- offline (unfused) two-side ABFT around the plain
// transform: the comparison baseline for the fused kernels (Sec. 2.2 "offline
// FT-FFT", Sec. 5.2).  The checksums are computed by kernels of their own, as
// a library-based scheme computes them with matrix-vector products over the
// batch, so the inputs and the outputs are read from HBM a second time:
//   1. input pass:  p_b = a^T x_b and nu_b = |x_b|^2 per signal, and the
//                   right-side sum x_s = sum of the group's inputs (groups of
//                   kOfflineT consecutive signals) written to a workspace;
//   2. the plain transform of x, and of the x_s rows (W x_s);
//   3. output pass: q_b = e^T y_b per signal (internal domain);
//   4. check:       signal b is faulty when |q_b - p_b| > tau_b;
//   5. fix:         a group with one faulty signal b* rebuilds it as
//                   y_b* = W x_s - sum_{b != b*} y_b (Eq. 5); more than one
//                   faulty signal in a group is counted uncorrectable.
// Every step is a kernel launch on the caller's stream; nothing waits on the
// host, so the call can be captured like the fused one.
#include <hip/hip_runtime.h>

#include "tfft_kernels.hpp"
#include "tfft_offline.hpp"

namespace tfft {

namespace {

constexpr int kOffThreads = 256;
constexpr int kOffEPT = 4;    // elements per thread and signal in the passes

// encoding vector e_n = w_M^(n mod M) (M = 3, or 5 when 3 | N)
template <class V> __device__ __forceinline__ V enc_e(long long n, int M) {
    if (M == 3) return wM<V, 3>((int)(n % 3));
    return wM<V, 5>((int)(n % 5));
}

// Input or output pass over groups of kOfflineT signals.  Thread (tile, tid)
// handles elements n = tile * kOffThreads * kOffEPT + r * kOffThreads + tid
// of every signal of its group: reads each value once, adds w_n v to the
// signal's checksum (w = the left vector a for inputs, e for outputs), |v|^2
// to its energy (inputs) and v to the group's right-side sum (inputs).  The
// per-signal partials are reduced over the workgroup and added atomically.
// The per-signal totals are double in both precisions: each workgroup adds
// its partial atomically, in no fixed order, and fp32 totals built that way
// over 2^20 elements carry rounding of the order of the threshold itself.
template <class V, bool IN>
__global__ __launch_bounds__(kOffThreads) void k_offline_pass(const V* __restrict__ z, long long N, long long batch,
                                                              const V* __restrict__ left, int M, int conj,
                                                              typename RealOf<V>::type inv_scale, double2* __restrict__ cs,
                                                              double* __restrict__ nu, V* __restrict__ xs,
                                                              long long tiles) {
    using R = typename RealOf<V>::type;
    constexpr int T = kOfflineT;
    __shared__ R red[2 * T + T][kOffThreads / kWave];
    const long long grp = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int tid = threadIdx.x;
    V acc[T];
    R en[T];
#pragma unroll
    for (int b = 0; b < T; ++b) { acc[b] = V{0, 0}; en[b] = 0; }
#pragma unroll
    for (int r = 0; r < kOffEPT; ++r) {
        const long long n = tile * (kOffThreads * kOffEPT) + (long long)r * kOffThreads + tid;
        if (n >= N) continue;
        V w = IN ? left[n] : enc_e<V>(n, M);
        V s = V{0, 0};
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const long long sig = grp * T + b;
            if (sig >= batch) continue;
            V v = z[sig * N + n];
            if (conj) v.y = -v.y;
            if (!IN) v = V{v.x * inv_scale, v.y * inv_scale};
            acc[b] = cmac(acc[b], w, v);
            if (IN) {
                en[b] = fmad(v.x, v.x, fmad(v.y, v.y, en[b]));
                s = cadd(s, v);
            }
        }
        if (IN) xs[grp * N + n] = s;
    }
    // workgroup reduction of the T checksums (and energies)
    const int lane = tid % kWave, wave = tid / kWave;
#pragma unroll
    for (int b = 0; b < T; ++b) {
        const R a0 = xor_reduce<1, kWave, OpAdd>(acc[b].x);
        const R a1 = xor_reduce<1, kWave, OpAdd>(acc[b].y);
        const R a2 = IN ? xor_reduce<1, kWave, OpAdd>(en[b]) : (R)0;
        if (lane == 0) {
            red[3 * b][wave] = a0;
            red[3 * b + 1][wave] = a1;
            red[3 * b + 2][wave] = a2;
        }
    }
    __syncthreads();
    if (tid < 3 * T) {
        R s = 0;
#pragma unroll
        for (int w = 0; w < kOffThreads / kWave; ++w) s += red[tid][w];
        const int b = tid / 3, k = tid % 3;
        const long long sig = grp * T + b;
        if (sig < batch) {
            if (k < 2) atomicAdd(reinterpret_cast<double*>(cs + sig) + k, (double)s);
            else if (IN) atomicAdd(&nu[sig], (double)s);
        }
    }
}

// per-signal check; flags[b] = 1 for a faulty signal, counts detected
__global__ void k_offline_check(const double2* __restrict__ p, const double2* __restrict__ q,
                                const double* __restrict__ nu, long long batch, double tau_coef,
                                int* __restrict__ flags, FtCounts* counts) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double dx = q[b].x - p[b].x, dy = q[b].y - p[b].y;
    const double tau = tau_coef * __builtin_sqrt(nu[b]);
    const bool checked = nu[b] == nu[b] && nu[b] < (double)INFINITY;
    const bool bad = checked && !(__builtin_sqrt(dx * dx + dy * dy) <= tau);
    flags[b] = bad ? 1 : 0;
    if (bad) {
        atomicAdd(&counts->detected, 1ull);
        atomicExch(&counts->last_signal, (unsigned long long)b);
    }
}

// Rebuild the faulty signal of each group from the right-side sums:
// y_b* = scale cj(W x_s - sum_{b != b*} y_b / scale).  Workgroups of a group
// without a fault return at once.
template <class V>
__global__ __launch_bounds__(kOffThreads) void k_offline_fix(V* __restrict__ y, const V* __restrict__ wxs, long long N,
                                                             long long batch, const int* __restrict__ flags, int conj,
                                                             typename RealOf<V>::type scale, long long tiles,
                                                             FtCounts* counts) {
    using R = typename RealOf<V>::type;
    constexpr int T = kOfflineT;
    const long long grp = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    int nbad = 0, bstar = -1;
    for (int b = 0; b < T; ++b) {
        const long long sig = grp * T + b;
        if (sig < batch && flags[sig]) { ++nbad; bstar = b; }
    }
    if (nbad == 0) return;
    if (nbad > 1) {
        if (tile == 0 && threadIdx.x == 0) {
            atomicAdd(&counts->uncorrectable, (unsigned long long)nbad);
        }
        return;
    }
    if (tile == 0 && threadIdx.x == 0) atomicAdd(&counts->rebuilt, 1ull);
    for (int r = 0; r < kOffEPT; ++r) {
        const long long n = tile * (kOffThreads * kOffEPT) + (long long)r * kOffThreads + threadIdx.x;
        if (n >= N) continue;
        V acc = wxs[grp * N + n];
        for (int b = 0; b < T; ++b) {
            const long long sig = grp * T + b;
            if (sig >= batch || b == bstar) continue;
            V v = y[sig * N + n];
            if (conj) v.y = -v.y;
            acc = V{acc.x - v.x / scale, acc.y - v.y / scale};
        }
        if (conj) acc.y = -acc.y;
        y[(grp * T + bstar) * N + n] = V{acc.x * scale, acc.y * scale};
    }
}

__global__ void k_offline_zero(double2* p, double* nu, long long batch) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) {
        p[b] = double2{0, 0};
        p[batch + b] = double2{0, 0};
        nu[b] = 0;
    }
}

}  // namespace

template <class V>
hipError_t offline_launch(const OfflineArgs& o, hipStream_t s, int step) {
    using R = typename RealOf<V>::type;
    const V* x = static_cast<const V*>(o.x);
    V* y = static_cast<V*>(o.y);
    double2* cs = static_cast<double2*>(o.cs);   // p (batch), then q (batch)
    double* nu = static_cast<double*>(o.nu);
    V* xs = static_cast<V*>(o.xs);
    const long long tiles = (o.N + kOffThreads * kOffEPT - 1) / (kOffThreads * kOffEPT);
    const long long groups = (o.batch + kOfflineT - 1) / kOfflineT;
    const unsigned g1 = (unsigned)((o.batch + 255) / 256);
    FtCounts* counts = reinterpret_cast<FtCounts*>(o.counts);
    switch (step) {
        case 0:
            hipLaunchKernelGGL(k_offline_zero, dim3(g1), dim3(256), 0, s, cs, nu, o.batch);
            hipLaunchKernelGGL((k_offline_pass<V, true>), dim3((unsigned)(groups * tiles)), dim3(kOffThreads), 0, s,
                               x, o.N, o.batch, static_cast<const V*>(o.left), o.M, o.conj, (R)1, cs, nu, xs, tiles);
            break;
        case 1:
            hipLaunchKernelGGL((k_offline_pass<V, false>), dim3((unsigned)(groups * tiles)), dim3(kOffThreads), 0, s,
                               (const V*)y, o.N, o.batch, static_cast<const V*>(o.left), o.M, o.conj,
                               (R)(1.0 / o.scale), cs + o.batch, nu, xs, tiles);
            hipLaunchKernelGGL(k_offline_check, dim3(g1), dim3(256), 0, s, (const double2*)cs,
                               (const double2*)(cs + o.batch), (const double*)nu, o.batch, o.tau_coef,
                               static_cast<int*>(o.flags), counts);
            break;
        default:
            hipLaunchKernelGGL(k_offline_fix<V>, dim3((unsigned)(groups * tiles)), dim3(kOffThreads), 0, s, y,
                               (const V*)xs, o.N, o.batch, (const int*)o.flags, o.conj, (R)o.scale, tiles, counts);
            break;
    }
    return hipGetLastError();
}

template hipError_t offline_launch<float2>(const OfflineArgs&, hipStream_t, int);
template hipError_t offline_launch<double2>(const OfflineArgs&, hipStream_t, int);

}  // namespace tfft
