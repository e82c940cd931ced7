// Variant 1 of the fp32 single-pass kernels of 512..8192 points: 8 elements
// per lane and radix-8 stages.  Twice the lanes per signal and half the data
// registers per lane, so the ABFT kernels keep more waves resident (four per
// SIMD) at the price of one more exchange through LDS.  The autotuner
// chooses per length and mode.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32_single_e8(std::vector<KernelEntry>& out) {
    add_plan<float2, kSingle, 512, 8, 4, 4, 8, 8, 8>(out, 0, 1);
    add_plan<float2, kSingle, 1024, 8, 4, 4, 2, 8, 8, 8>(out, 0, 1);
    add_plan<float2, kSingle, 2048, 8, 4, 4, 4, 8, 8, 8>(out, 0, 1);
    add_plan<float2, kSingle, 4096, 8, 4, 4, 8, 8, 8, 8>(out, 0, 1);
    add_plan<float2, kSingle, 8192, 8, 4, 4, 2, 8, 8, 8, 8>(out, 0, 1);
}

}  // namespace tfft
