// fp32 column/row pass kernels for N = N1 * N2 > 8192: sub-lengths 64..2048,
// E = 16, 16 sub-signals per tile (128-byte contiguous accesses) up to 512
// points, then 8 and 4 so that a workgroup stays at 512 lanes; neighbouring
// tiles complete each other's cache lines in the same L2.
#include "tfft_registry.hpp"

namespace tfft {

template <int KIND> static void add_kind(std::vector<KernelEntry>& out) {
    add_plan<float2, KIND, 64, 16, 16, 0, 4, 16>(out, 0);
    add_plan<float2, KIND, 128, 16, 16, 0, 8, 16>(out, 0);
    add_plan<float2, KIND, 256, 16, 16, 0, 16, 16>(out, 0);
    add_plan<float2, KIND, 512, 16, 16, 0, 2, 16, 16>(out, 0);
    add_plan<float2, KIND, 1024, 16, 8, 0, 4, 16, 16>(out, 0);
    add_plan<float2, KIND, 2048, 16, 4, 0, 8, 16, 16>(out, 0);
}

void register_fp32_tiles(std::vector<KernelEntry>& out) {
    add_kind<kColPass>(out);
    add_kind<kRowPass>(out);
    register_fp32_tiles_narrow(out);
    register_fp32_tiles_e8(out);
    register_fp32_tiles_wide(out);
}

}  // namespace tfft
