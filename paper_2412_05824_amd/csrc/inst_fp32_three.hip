// fp32 kernels of the second and third pass of three-pass transforms
// (N = N1 N2 N3 > 2^22): column pass B over rows of length N2 N3 with the
// outer twiddle at load, 16 columns per tile; row pass C over (signal, k2)
// pairs, 8 rows k1 per tile so that its transposed outputs k1 + N1 (k2 +
// N2 k3) leave in 64-byte runs.  Pass A is the regular column pass.
#include "tfft_registry.hpp"

namespace tfft {

void register_fp32_three(std::vector<KernelEntry>& out) {
    add_plan<float2, kColPass3, 256, 16, 16, 0, 16, 16>(out, 0);
    add_plan<float2, kColPass3, 512, 16, 16, 0, 2, 16, 16>(out, 0);
    add_plan<float2, kRowPass3, 256, 16, 8, 0, 16, 16>(out, 0);
    add_plan<float2, kRowPass3, 512, 16, 8, 0, 2, 16, 16>(out, 0);
    // variant 1: 16 rows per tile, 128-byte output runs
    add_plan<float2, kRowPass3, 256, 16, 16, 0, 16, 16>(out, 0, 1);
    add_plan<float2, kRowPass3, 512, 16, 16, 0, 2, 16, 16>(out, 0, 1);
}

}  // namespace tfft
