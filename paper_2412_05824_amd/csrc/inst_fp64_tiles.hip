// fp64 column/row pass kernels for N = N1 * N2 > 4096: sub-lengths 64..1024,
// E = 8, 8 sub-signals per tile (128-byte contiguous accesses), 4 for the
// 1024-point sub-length so that a workgroup stays at 512 lanes.
#include "tfft_registry.hpp"

namespace tfft {

template <int KIND> static void add_kind(std::vector<KernelEntry>& out) {
    add_plan<double2, KIND, 64, 8, 8, 0, 8, 8>(out, 1);
    add_plan<double2, KIND, 128, 8, 8, 0, 2, 8, 8>(out, 1);
    add_plan<double2, KIND, 256, 8, 8, 0, 4, 8, 8>(out, 1);
    add_plan<double2, KIND, 512, 8, 8, 0, 8, 8, 8>(out, 1);
    add_plan<double2, KIND, 1024, 8, 4, 0, 2, 8, 8, 8>(out, 1);
}

void register_fp64_tiles(std::vector<KernelEntry>& out) {
    add_kind<kColPass>(out);
    add_kind<kRowPass>(out);
}

}  // namespace tfft
