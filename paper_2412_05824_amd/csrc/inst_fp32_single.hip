// Single-pass fp32 kernels: E = 16 elements per lane, radix-16 stages after
// one smaller leading radix, 4 waves per workgroup for sub-wave slots, one
// LDS pad element per 16 (128-byte rows).
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32_single(std::vector<KernelEntry>& out) {
    add_plan<float2, kSingle, 64, 16, 4, 4, 4, 16>(out, 0);
    add_plan<float2, kSingle, 128, 16, 4, 4, 8, 16>(out, 0);
    add_plan<float2, kSingle, 256, 16, 4, 4, 16, 16>(out, 0);
    add_plan<float2, kSingle, 512, 16, 4, 4, 2, 16, 16>(out, 0);
    add_plan<float2, kSingle, 1024, 16, 4, 4, 4, 16, 16>(out, 0);
    add_plan<float2, kSingle, 2048, 16, 4, 4, 8, 16, 16>(out, 0);
    add_plan<float2, kSingle, 4096, 16, 4, 4, 16, 16, 16>(out, 0);
    add_plan<float2, kSingle, 8192, 16, 4, 4, 2, 16, 16, 16>(out, 0);
    register_fp32_single_e8(out);
    register_fp32_single_stream(out);
    register_fp32_single_16k(out);
}

}  // namespace tfft
