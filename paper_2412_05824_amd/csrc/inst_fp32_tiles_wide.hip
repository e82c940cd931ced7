// fp32 column and row passes of 1024 and 2048 points with wide tiles: 16
// and 8 sub-signals per workgroup, so that column reads and transposed row
// stores move 128- and 64-byte runs; variant 3 keeps E = 16 (1024 threads),
// variant 4 takes E = 32 (512 threads, two butterflies per lane per stage).
#include "tfft_registry.hpp"

namespace tfft {

template <int KIND> static void add_wide(std::vector<KernelEntry>& out) {
    add_plan<float2, KIND, 1024, 16, 16, 0, 4, 16, 16>(out, 0, 3);
    add_plan<float2, KIND, 2048, 16, 8, 0, 8, 16, 16>(out, 0, 3);
    add_plan<float2, KIND, 1024, 32, 16, 0, 4, 16, 16>(out, 0, 4);
    add_plan<float2, KIND, 2048, 32, 8, 0, 8, 16, 16>(out, 0, 4);
}

void register_fp32_tiles_wide(std::vector<KernelEntry>& out) {
    add_wide<kColPass>(out);
    add_wide<kRowPass>(out);
}

}  // namespace tfft
