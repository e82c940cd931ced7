// Variant 1 of the fp32 column/row passes of 512..2048 points: half the
// sub-signals per tile (8, 4, 2), so a workgroup has 256 lanes and two or
// three fit a CU beside the registers of the ABFT kernels, at the price of
// shorter contiguous segments.  The autotuner chooses per length and mode.
#include "tfft_registry.hpp"

namespace tfft {

template <int KIND> static void add_narrow(std::vector<KernelEntry>& out) {
    add_plan<float2, KIND, 512, 16, 8, 0, 2, 16, 16>(out, 0, 1);
    add_plan<float2, KIND, 1024, 16, 4, 0, 4, 16, 16>(out, 0, 1);
    add_plan<float2, KIND, 2048, 16, 2, 0, 8, 16, 16>(out, 0, 1);
}

void register_fp32_tiles_narrow(std::vector<KernelEntry>& out) {
    add_narrow<kColPass>(out);
    add_narrow<kRowPass>(out);
}

}  // namespace tfft
