// fp32 single-pass kernels of 16384 points (streaming form: e^T W read from
// the cached table, the signal alone in 136 KiB of padded LDS, one
// workgroup per CU): variant 0 E = 16 (1024 lanes), variant 1 E = 32 (512
// lanes, two butterflies per lane per stage).  The autotuner weighs them
// against the two-pass splits.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32_single_16k(std::vector<KernelEntry>& out) {
    add_plan<float2, kSingle, 16384, 16, 1, 4, 4, 16, 16, 16>(out, 0, 0);
    add_plan<float2, kSingle, 16384, 32, 1, 4, 4, 16, 16, 16>(out, 0, 1);
}

}  // namespace tfft
