// Streaming fp64 single-pass kernels of 1024..4096 points (variant 1): the
// checking form reads e^T W from the cached table (no resident staging) and
// is held to the occupancy its LDS allows, spilling only on the error path.
// Variant 2 of 1024 points: E = 4 (four waves per signal, radix-4 stages),
// 121 VGPRs with ABFT, four waves per SIMD without spills.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp64_single_stream(std::vector<KernelEntry>& out) {
    add_plan<double2, kSingle, 1024, 8, 1, 3, 2, 8, 8, 8>(out, 1, 1);
    add_plan<double2, kSingle, 2048, 8, 1, 3, 4, 8, 8, 8>(out, 1, 1);
    add_plan<double2, kSingle, 4096, 8, 1, 3, 8, 8, 8, 8>(out, 1, 1);
    add_plan<double2, kSingle, 1024, 4, 1, 3, 4, 4, 4, 4, 4>(out, 1, 2);
}

}  // namespace tfft
