// tfft_registry.hpp -- host-side description of every compiled kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "tfft_kernels.hpp"

namespace tfft {

using LaunchFn = hipError_t (*)(const void* x, void* y, const void* kargs, long long grid,
                                hipStream_t stream);

struct KernelEntry {
    int precision;          // 0 fp32, 1 fp64
    int N;                  // transform length
    int ft;                 // 0 off, 1 detect, 2 correct
    int E, P, threads;      // elements per lane, lanes per slot, lanes per workgroup
    int slots_per_block;    // signals per workgroup per transaction
    int n_stages;
    int radices[8];
    LaunchFn launch;
};

template <class V, class PL, int FT, int... Rs>
hipError_t launch_single(const void* x, void* y, const void* ka, long long grid, hipStream_t s) {
    const KArgs<V>& a = *static_cast<const KArgs<V>*>(ka);
    hipLaunchKernelGGL((k_single<V, PL, FT, Rs...>), dim3((unsigned)grid), dim3(PL::THREADS), 0, s,
                       static_cast<const V*>(x), static_cast<V*>(y), a);
    return hipGetLastError();
}

template <class V, class PL, int FT, int... Rs> KernelEntry make_single_entry(int precision) {
    KernelEntry e{};
    e.precision = precision;
    e.N = PL::N;
    e.ft = FT;
    e.E = PL::E;
    e.P = PL::P;
    e.threads = PL::THREADS;
    e.slots_per_block = PL::SLOTS;
    const int rs[] = {Rs...};
    e.n_stages = (int)sizeof...(Rs);
    for (int i = 0; i < e.n_stages; ++i) e.radices[i] = rs[i];
    e.launch = &launch_single<V, PL, FT, Rs...>;
    return e;
}

template <class V, int N, int E, int WPB, int B, int... Rs>
void add_single(std::vector<KernelEntry>& out, int precision) {
    using PL = Plan<N, E, WPB, B, Rs...>;
    out.push_back(make_single_entry<V, PL, 0, Rs...>(precision));
    out.push_back(make_single_entry<V, PL, 1, Rs...>(precision));
    out.push_back(make_single_entry<V, PL, 2, Rs...>(precision));
}

void register_fp32(std::vector<KernelEntry>& out);
void register_fp64(std::vector<KernelEntry>& out);

}  // namespace tfft
