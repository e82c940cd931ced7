// Streaming fp32 single-pass kernels: the checking form reads e^T W (its
// cotangent form) from the cached table instead of staging it in LDS, with
// no resident loop.  8192 points: the 64 KiB exchange buffer is all a
// workgroup holds and two workgroups share a CU; variant 2: E = 16 (8 waves
// per signal), variant 3: E = 32 (4 waves, two butterflies per lane per
// stage).  1024-4096 points, variant 2: E = 8, five waves per SIMD.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32_single_stream(std::vector<KernelEntry>& out) {
    add_plan<float2, kSingle, 8192, 16, 1, 4, 2, 16, 16, 16>(out, 0, 2);
    add_plan<float2, kSingle, 8192, 32, 1, 4, 2, 16, 16, 16>(out, 0, 3);
    add_plan<float2, kSingle, 1024, 8, 1, 4, 2, 8, 8, 8>(out, 0, 2);
    add_plan<float2, kSingle, 2048, 8, 1, 4, 4, 8, 8, 8>(out, 0, 2);
    add_plan<float2, kSingle, 4096, 8, 1, 4, 8, 8, 8, 8>(out, 0, 2);
}

}  // namespace tfft
