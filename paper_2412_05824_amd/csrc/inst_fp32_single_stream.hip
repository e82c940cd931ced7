// Streaming fp32 single-pass kernels of 8192 points: the checking form reads
// e^T W from the cached table instead of staging it in LDS, so the 64 KiB
// exchange buffer is all a workgroup holds and two workgroups share a CU.
// Variant 2: E = 16 (8 waves per signal); variant 3: E = 32 (4 waves, two
// butterflies per lane per stage).
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32_single_stream(std::vector<KernelEntry>& out) {
    add_plan<float2, kSingle, 8192, 16, 1, 4, 2, 16, 16, 16>(out, 0, 2);
    add_plan<float2, kSingle, 8192, 32, 1, 4, 2, 16, 16, 16>(out, 0, 3);
}

}  // namespace tfft
