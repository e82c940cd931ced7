// tfft_registry.hpp -- host-side description of every compiled kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "tfft_kernels.hpp"

namespace tfft {

using LaunchFn = hipError_t (*)(const void* x, void* y, const void* kargs, long long grid,
                                hipStream_t stream);

constexpr int kMaxStages = 14;   // radix stages a registered plan may have

struct KernelEntry {
    int precision;          // 0 fp32, 1 fp64
    int kind;               // kSingle, kColPass, kRowPass, kColPass3, kRowPass3
    int Ns;                 // (sub-)transform length
    int ft;                 // 0 off, 1 detect, 2 correct, 3 correct in place, 4 thread-level
    int E, P, threads;      // elements per lane, lanes per slot, lanes per workgroup
    int slots_per_block;    // sub-signals per workgroup per transaction
    int n_stages;
    int radices[kMaxStages];
    LaunchFn launch;
    int ragged_id;          // index in the ragged plan list (-1: regular plan)
    int variant;            // plans of one (kind, Ns): 0 default, 1.. alternatives
    int tx_max;             // per-transaction checking: most transactions per group
    int cot;                // 1: reads the left vector in cotangent form (KArgs::cot)
};

// grid: workgroups' worth of work.  Resident kernels launch at most as many
// workgroups as the device holds at once and loop over the rest.
template <class V, class PL, int FT, bool IND, int... Rs>
hipError_t launch_fft(const void* x, void* y, const void* ka, long long grid, hipStream_t s) {
    KArgs<V> a = *static_cast<const KArgs<V>*>(ka);
    a.nblk = grid;
    long long g = grid;
    if constexpr (kResident<V, PL, kGroupFt<FT>, IND>) {
        static const int per_cu = [] {
            int n = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fft<V, PL, FT, IND, Rs...>, PL::THREADS, 0) !=
                    hipSuccess || n < 1)
                n = 1;
            return n;
        }();
        int dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        const long long cap = (long long)per_cu * (cus > 0 ? cus : 1);
        if (g > cap) g = cap;
    }
    hipLaunchKernelGGL((k_fft<V, PL, FT, IND, Rs...>), dim3((unsigned)g), dim3(PL::THREADS), 0, s,
                       static_cast<const V*>(x), static_cast<V*>(y), a);
    return hipGetLastError();
}

template <class V, class PL, int FT, bool IND, int... Rs> KernelEntry make_entry(int precision) {
    KernelEntry e{};
    e.precision = precision;
    e.kind = PL::KIND;
    e.Ns = PL::Ns;
    e.ft = FT;
    e.E = PL::E;
    e.P = PL::P;
    e.threads = PL::THREADS;
    e.slots_per_block = PL::SLOTS;
    const int rs[] = {Rs...};
    static_assert(sizeof...(Rs) <= kMaxStages, "too many stages for the registry");
    e.n_stages = (int)sizeof...(Rs);
    for (int i = 0; i < e.n_stages; ++i) e.radices[i] = rs[i];
    e.launch = &launch_fft<V, PL, FT, IND, Rs...>;
    e.ragged_id = -1;
    e.variant = 0;
    e.tx_max = Geo<V, PL, IND>::TX_MAX;
    e.cot = kCotLeft<V, PL, kGroupFt<FT>, IND> ? 1 : 0;
    return e;
}

// register the ABFT modes of one plan (in-place correction: single pass only;
// the passes of a two-pass transform never overwrite their own inputs)
template <class V, int KIND, int Ns, int E, int WC, int B, int... Rs>
void add_plan(std::vector<KernelEntry>& out, int precision, int variant = 0) {
    using PL = Plan<KIND, Ns, E, WC, B, Rs...>;
    KernelEntry e[5] = {make_entry<V, PL, 0, false, Rs...>(precision),
                        make_entry<V, PL, 1, false, Rs...>(precision),
                        make_entry<V, PL, 2, false, Rs...>(precision), {}, {}};
    int n = 3;
    // single pass: the in-place correcting form, and thread-level ABFT
    if constexpr (KIND == kSingle) {
        e[n++] = make_entry<V, PL, 3, false, Rs...>(precision);
        e[n++] = make_entry<V, PL, 4, false, Rs...>(precision);
    }
    for (int i = 0; i < n; ++i) {
        e[i].variant = variant;
        out.push_back(e[i]);
    }
}

void register_fp32_single(std::vector<KernelEntry>& out);
void register_fp32_single_e8(std::vector<KernelEntry>& out);
void register_fp32_single_stream(std::vector<KernelEntry>& out);
void register_fp32_single_16k(std::vector<KernelEntry>& out);
void register_fp32_tiles(std::vector<KernelEntry>& out);
void register_fp32_tiles_narrow(std::vector<KernelEntry>& out);
void register_fp32_tiles_e8(std::vector<KernelEntry>& out);
void register_fp32_tiles_wide(std::vector<KernelEntry>& out);
void register_fp64_single(std::vector<KernelEntry>& out);
void register_fp64_single_stream(std::vector<KernelEntry>& out);
void register_fp64_single_8k(std::vector<KernelEntry>& out);
void register_fp64_tiles(std::vector<KernelEntry>& out);
void register_fp32_three(std::vector<KernelEntry>& out);
// the stepwise study's radix-2 plans (not in the route registry) and its
// per-stage kernel
void register_fp32_stepwise(std::vector<KernelEntry>& out);
hipError_t radix2_stage_launch(const void* x, void* y, long long N, long long batch, long long L,
                               const void* hi, const void* lo, int bits, int conj, float scale,
                               hipStream_t s);

}  // namespace tfft
