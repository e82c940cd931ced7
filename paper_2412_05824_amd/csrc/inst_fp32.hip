// Single-pass fp32 kernels: E = 16 elements per lane, radix-16 stages with one
// smaller leading radix, 4 waves per workgroup for sub-wave slots, XOR swizzle
// over 16-element (128-byte) LDS rows.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32(std::vector<KernelEntry>& out) {
    add_single<float2, 64, 16, 4, 4, 4, 16>(out, 0);
    add_single<float2, 128, 16, 4, 4, 8, 16>(out, 0);
    add_single<float2, 256, 16, 4, 4, 16, 16>(out, 0);
    add_single<float2, 512, 16, 4, 4, 2, 16, 16>(out, 0);
    add_single<float2, 1024, 16, 4, 4, 4, 16, 16>(out, 0);
    add_single<float2, 2048, 16, 4, 4, 8, 16, 16>(out, 0);
    add_single<float2, 4096, 16, 4, 4, 16, 16, 16>(out, 0);
    add_single<float2, 8192, 16, 4, 4, 2, 16, 16, 16>(out, 0);
}

}  // namespace tfft
