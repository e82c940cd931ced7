// Variant 2 of the fp32 column/row passes of 64..512 points: 8 elements per
// lane (radix-8 stages) and 256 lanes per workgroup, the ABFT kernels' lighter
// register footprint (four waves per SIMD) against shorter contiguous
// segments at 256 and 512 points.  The autotuner chooses per length and mode.
#include "tfft_registry.hpp"

namespace tfft {

template <int KIND> static void add_e8(std::vector<KernelEntry>& out) {
    add_plan<float2, KIND, 64, 8, 32, 0, 8, 8>(out, 0, 2);
    add_plan<float2, KIND, 128, 8, 16, 0, 2, 8, 8>(out, 0, 2);
    add_plan<float2, KIND, 256, 8, 8, 0, 4, 8, 8>(out, 0, 2);
    add_plan<float2, KIND, 512, 8, 4, 0, 8, 8, 8>(out, 0, 2);
}

void register_fp32_tiles_e8(std::vector<KernelEntry>& out) {
    add_e8<kColPass>(out);
    add_e8<kRowPass>(out);
}

}  // namespace tfft
