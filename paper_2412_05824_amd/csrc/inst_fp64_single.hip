// Single-pass fp64 kernels: E = 8 elements per lane, radix-8 stages after one
// smaller leading radix, XOR swizzle over 8-element (128-byte) LDS rows.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp64_single(std::vector<KernelEntry>& out) {
    add_plan<double2, kSingle, 64, 8, 4, 3, 8, 8>(out, 1);
    add_plan<double2, kSingle, 128, 8, 4, 3, 2, 8, 8>(out, 1);
    add_plan<double2, kSingle, 256, 8, 4, 3, 4, 8, 8>(out, 1);
    add_plan<double2, kSingle, 512, 8, 4, 3, 8, 8, 8>(out, 1);
    add_plan<double2, kSingle, 1024, 8, 4, 3, 2, 8, 8, 8>(out, 1);
    add_plan<double2, kSingle, 2048, 8, 4, 3, 4, 8, 8, 8>(out, 1);
    add_plan<double2, kSingle, 4096, 8, 4, 3, 8, 8, 8, 8>(out, 1);
    register_fp64_single_stream(out);
    register_fp64_single_8k(out);
}

}  // namespace tfft
