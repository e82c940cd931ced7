// fp64 single-pass kernel of 8192 points (streaming form: e^T W read from
// the cached table, the signal alone in 136 KiB of padded LDS, 512 lanes of
// E = 16, one workgroup per CU).  The autotuner weighs it against the
// two-pass splits.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp64_single_8k(std::vector<KernelEntry>& out) {
    add_plan<double2, kSingle, 8192, 16, 1, 3, 2, 16, 16, 16>(out, 1, 0);
}

}  // namespace tfft
