// The persistent ragged kernel with ABFT mode 2.
#include "tfft_ragged_kernel.hpp"

namespace tfft {

RaggedKernel ragged_kernel_ft2(int waves) {
    return waves == 3 ? make_ragged_kernel<2, true>() : make_ragged_kernel<2, false>();
}

}  // namespace tfft
