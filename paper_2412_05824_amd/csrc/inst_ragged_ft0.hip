// The persistent ragged kernel with ABFT mode 0.
#include "tfft_ragged_kernel.hpp"

namespace tfft {

RaggedKernel ragged_kernel_ft0(int waves) {
    (void)waves;   // already at four workgroups per CU
    return make_ragged_kernel<0, false>();
}

}  // namespace tfft
